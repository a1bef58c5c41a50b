// Pair schedules of the exchange passes (host code).
//
// A system's pairs i <= j are evaluated in tile pairs of `rows` orbitals (I)
// x `tile` orbitals (J), described by TileDesc.  A batch is a set of tile
// pairs that touch disjoint orbitals, so that the workgroups of one launch
// never update the same orbital's K psi; the three passes of a batch run
// back to back and batches run in order, which fixes the summation order.
// Each tile pair owns rows x tile / 2 consecutive pair-grid slots of its
// batch (two pairs (a, 2g) and (a, 2g + 1) share a complex grid); `active`
// lists the slots that carry at least one evaluated pair.
#pragma once

#include <utility>
#include <vector>

#include "hfx_internal.hpp"

namespace hfx {

struct Batch {
  int tile_off, n_tiles;      // tile pairs [tile_off, tile_off + n_tiles)
  int active_off, n_active;   // slots [active_off, active_off + n_active) of `active`
  long long part_base;        // first energy partial (one per tile pair and brick)
};

// What a schedule is built for.
struct ScheduleShape {
  int n_orb;       // orbitals of the system
  int tile;        // J orbitals per tile pair (T)
  int rows;        // I orbitals per tile pair (R: a multiple of T, at most kMaxRows)
  int bricks;      // pencil workgroups per tile pair (one energy partial each)
  int shard = 0;   // virtual group g of `shards`: rounds (screened: batches) r with
  int shards = 1;  //   r % shards == g
};

struct Schedule {
  int tiles_per_batch = 1;  // most tile pairs in a batch
  int slots_per_batch = 0;  // pair-grid slots of the batch buffer
  std::vector<TileDesc> tiles;
  std::vector<int> active;  // slot of every transformed pair grid, batch by batch
  std::vector<Batch> batches;
  long long n_partials = 0;
};

// Round-robin (circle method) rounds of nb blocks: each round lists block
// pairs (I, J), I <= J, in which no block appears twice; together the rounds
// list every pair once (the diagonal pairs (B, B) included).
std::vector<std::vector<std::pair<int, int>>> tile_rounds(int nb);

// Every pair i <= j.  Batches of at most tiles_cap tile pairs when
// tiles_cap > 0 (else enough for about 4096 pencil workgroups).
Schedule build_schedule(const ScheduleShape& sh, long long tiles_cap);

// Orbital order for screening: runs of `tile` strongly overlapping orbitals
// (greedy clustering on the symmetric n x n overlap a over the kept pairs).
std::vector<int> cluster_order(int n, int tile, const std::vector<double>& a,
                               const std::vector<unsigned char>& keep);

// Bit of pair (row a, column b) in a tile pair's keep mask.
bool keep_bit(const TileDesc& td, int a, int b);

// The pairs kept by keep (n x n, symmetric, original orbital indices) over
// the order perm (position -> orbital), in batches that fit slots_per_batch
// pair-grid slots.
Schedule build_screened_schedule(const ScheduleShape& sh, int slots_per_batch,
                                 const std::vector<unsigned char>& keep,
                                 const std::vector<int>& perm);

}  // namespace hfx
