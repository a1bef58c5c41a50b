// Pair schedules of the exchange passes (host code, no device calls):
// which tile pairs run, in which batches, on which pair-grid slots.  Kept
// apart from the C ABI so that the CPU tests can check them.
#include "schedule.hpp"

#include <algorithm>

namespace hfx {

// Round-robin (circle method) schedule of orbital blocks: each round lists
// block pairs (I, J), I <= J, in which no block appears twice.
std::vector<std::vector<std::pair<int, int>>> tile_rounds(int nb) {
  std::vector<std::vector<std::pair<int, int>>> rounds;
  if (nb == 1) {
    rounds.push_back({{0, 0}});
    return rounds;
  }
  const bool odd = nb % 2 == 1;
  const int n = odd ? nb + 1 : nb;  // team nb is the dummy when odd
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[i] = i;
  for (int r = 0; r < n - 1; ++r) {
    std::vector<std::pair<int, int>> round;
    for (int i = 0; i < n / 2; ++i) {
      int a = pos[i], b = pos[n - 1 - i];
      if (odd && (a == nb || b == nb)) {
        const int c = a == nb ? b : a;
        round.push_back({c, c});  // diagonal tile of the block left without partner
      } else {
        round.push_back({std::min(a, b), std::max(a, b)});
      }
    }
    rounds.push_back(round);
    // rotate all but the first position
    const int last = pos[n - 1];
    for (int i = n - 1; i > 1; --i) pos[i] = pos[i - 1];
    pos[1] = last;
  }
  if (!odd) {
    std::vector<std::pair<int, int>> diag;
    for (int b = 0; b < nb; ++b) diag.push_back({b, b});
    rounds.push_back(diag);
  }
  return rounds;
}

// Pair schedule of an unscreened plan.  Orbitals are grouped in blocks of R =
// sh.rows; the round-robin rounds pair the blocks, and block pair (BI, BJ) is
// cut into R / T tile pairs (all R rows of BI) x (tile q of BJ, T columns).
// The tile pairs of one round with the same q touch disjoint orbitals and form
// the batches (at most tiles_per_batch each); tile pairs sharing BI go to
// different batches, so no two workgroups of a launch update one orbital's
// K psi.  Inside a diagonal block only pairs i <= j are evaluated and rows
// below the tile's last column are dropped.  With R = T this is the plain
// T x T tiling.  Rows spread the J side (psi_J and K psi_J traffic) over R
// pairs per column instead of T.
Schedule build_schedule(const ScheduleShape& sh, long long tiles_cap) {
  // (rounds outside this plan's virtual group are skipped below)
  Schedule sp;
  const int T = sh.tile, R = sh.rows, n = sh.n_orb;
  const int sub = R / T;
  const int nb = (n + R - 1) / R;
  const auto rounds = tile_rounds(nb);
  const int br = sh.bricks;
  int tpb = std::max(1, (4096 + br - 1) / br);
  if (tiles_cap > 0) tpb = (int)std::min<long long>(tpb, tiles_cap);
  size_t max_round = 0;
  for (auto& r : rounds) max_round = std::max(max_round, r.size());
  tpb = std::min<int>(tpb, (int)max_round);
  sp.tiles_per_batch = tpb;
  sp.slots_per_batch = tpb * R * (T / 2);
  long long part = 0;
  for (size_t ri = 0; ri < rounds.size(); ++ri) {
    if ((int)(ri % (size_t)sh.shards) != sh.shard) continue;
    for (int q = 0; q < sub; ++q) {
      std::vector<TileDesc> group;
      for (const auto& bp : rounds[ri]) {
        TileDesc td{};
        td.i0 = bp.first * R;
        td.j0 = bp.second * R + q * T;
        if (td.j0 >= n) continue;
        td.nJ = std::min(T, n - td.j0);
        td.nI = std::min(R, n - td.i0);
        td.diag = bp.first == bp.second ? 1 : 0;
        td.joff = td.diag ? td.j0 - td.i0 : 0;
        if (td.diag) td.nI = std::min(td.nI, td.joff + td.nJ);
        td.keep0 = td.keep1 = td.keep2 = td.keep3 = ~0ull;
        group.push_back(td);
      }
      for (size_t s0 = 0; s0 < group.size(); s0 += tpb) {
        Batch b{};
        b.tile_off = (int)sp.tiles.size();
        b.active_off = (int)sp.active.size();
        b.part_base = part;
        const size_t e = std::min(group.size(), s0 + tpb);
        for (size_t k = s0; k < e; ++k) {
          TileDesc td = group[k];
          td.slot0 = (int)(k - s0) * R * (T / 2);
          for (int ia = 0; ia < td.nI; ++ia)
            for (int g = 0; g < T / 2; ++g) {
              const int b0 = 2 * g;
              if (b0 >= td.nJ) continue;
              if (td.diag && b0 + 1 + td.joff < ia) continue;  // both pairs below i = j
              sp.active.push_back(td.slot0 + ia * (T / 2) + g);
            }
          sp.tiles.push_back(td);
        }
        b.n_tiles = (int)sp.tiles.size() - b.tile_off;
        b.n_active = (int)sp.active.size() - b.active_off;
        part += (long long)b.n_tiles * br;
        sp.batches.push_back(b);
      }
    }
  }
  sp.n_partials = part;
  return sp;
}

// Orbital order of a screened plan: consecutive runs of `tile` orbitals that
// overlap strongly, so that whole tile pairs drop out.  Greedy clustering on
// the overlap measure A (symmetric, n x n): a cluster starts at the
// unassigned orbital with the fewest unassigned kept partners (the edge of
// what is left) and grows by the unassigned orbital with the largest summed
// A to the cluster's members.  Deterministic: ties go to the lower index.
std::vector<int> cluster_order(int n, int tile, const std::vector<double>& a,
                               const std::vector<unsigned char>& keep) {
  std::vector<int> deg(n, 0), order;
  std::vector<char> done(n, 0);
  std::vector<double> score(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (i != j && keep[(size_t)i * n + j]) ++deg[i];
  auto take = [&](int u) {
    done[u] = 1;
    order.push_back(u);
    for (int j = 0; j < n; ++j)
      if (j != u && keep[(size_t)j * n + u]) --deg[j];
  };
  while ((int)order.size() < n) {
    int seed = -1;
    for (int i = 0; i < n; ++i)
      if (!done[i] && (seed < 0 || deg[i] < deg[seed])) seed = i;
    take(seed);
    for (int j = 0; j < n; ++j) score[j] = a[(size_t)j * n + seed];
    for (int m = 1; m < tile && (int)order.size() < n; ++m) {
      int best = -1;
      for (int j = 0; j < n; ++j)
        if (!done[j] && (best < 0 || score[j] > score[best])) best = j;
      take(best);
      for (int j = 0; j < n; ++j) score[j] += a[(size_t)j * n + best];
    }
  }
  return order;
}

// Bit of pair (row a, column b) in a tile's keep mask.
bool keep_bit(const TileDesc& td, int a, int b) {
  return (keep_word(td, a >> 3) >> (8 * (a & 7) + b)) & 1ull;
}

// Schedule of a screened plan: the tile pairs of the unscreened schedule's
// shape (R rows x 8 columns over the reordered orbitals, i <= j inside a
// diagonal block) that keep at least one pair, each with the mask of its kept
// pairs, packed greedily (first fit, in (I, J, q) order) into batches whose
// tile pairs touch disjoint orbitals, as many per batch as the unscreened
// plan's pair-grid slots hold (so the workspace still fits).
Schedule build_screened_schedule(const ScheduleShape& sh, int slots_per_batch,
                                 const std::vector<unsigned char>& keep,
                                 const std::vector<int>& perm) {
  Schedule sp;
  const int T = sh.tile, R = sh.rows, n = sh.n_orb;
  const int nb = (n + R - 1) / R, nc = (n + T - 1) / T;
  const int br = sh.bricks;
  const int tpb = std::max(1, slots_per_batch / (R * (T / 2)));
  sp.tiles_per_batch = tpb;
  sp.slots_per_batch = slots_per_batch;
  std::vector<TileDesc> tps;
  for (int bi = 0; bi < nb; ++bi)
    for (int bj = bi; bj < nb; ++bj)
      for (int q = 0; q < R / T; ++q) {
        TileDesc td{};
        td.i0 = bi * R;
        td.j0 = bj * R + q * T;
        if (td.j0 >= n) continue;
        td.nJ = std::min(T, n - td.j0);
        td.nI = std::min(R, n - td.i0);
        td.diag = bi == bj ? 1 : 0;
        td.joff = td.diag ? td.j0 - td.i0 : 0;
        if (td.diag) td.nI = std::min(td.nI, td.joff + td.nJ);
        bool any = false;
        for (int a = 0; a < td.nI; ++a)
          for (int b = 0; b < td.nJ; ++b) {
            if (td.diag && b + td.joff < a) continue;
            if (keep[(size_t)perm[td.i0 + a] * n + perm[td.j0 + b]]) {
              unsigned long long* w[4] = {&td.keep0, &td.keep1, &td.keep2, &td.keep3};
              *w[a >> 3] |= 1ull << (8 * (a & 7) + b);
              any = true;
            }
          }
        if (any) tps.push_back(td);
      }
  // first fit; a tile pair occupies the T-orbital column tiles of its rows
  // and its column tile
  std::vector<std::vector<TileDesc>> batches;
  std::vector<std::vector<char>> used;
  for (const TileDesc& t : tps) {
    const int c0 = t.i0 / T, c1 = (t.i0 + t.nI - 1) / T, cj = t.j0 / T;
    auto fits = [&](const std::vector<char>& u) {
      for (int c = c0; c <= c1; ++c)
        if (u[c]) return false;
      return !u[cj];
    };
    size_t k = 0;
    for (; k < batches.size(); ++k)
      if ((int)batches[k].size() < tpb && fits(used[k])) break;
    if (k == batches.size()) {
      batches.emplace_back();
      used.emplace_back(nc, 0);
    }
    batches[k].push_back(t);
    for (int c = c0; c <= c1; ++c) used[k][c] = 1;
    used[k][cj] = 1;
  }
  long long part = 0;
  for (size_t k = 0; k < batches.size(); ++k) {
    if ((int)(k % (size_t)sh.shards) != sh.shard) continue;
    Batch b{};
    b.tile_off = (int)sp.tiles.size();
    b.active_off = (int)sp.active.size();
    b.part_base = part;
    for (size_t q = 0; q < batches[k].size(); ++q) {
      TileDesc td = batches[k][q];
      td.slot0 = (int)q * R * (T / 2);
      for (int ia = 0; ia < td.nI; ++ia)
        for (int g = 0; g < T / 2; ++g)
          if ((2 * g < td.nJ && keep_bit(td, ia, 2 * g)) ||
              (2 * g + 1 < td.nJ && keep_bit(td, ia, 2 * g + 1)))
            sp.active.push_back(td.slot0 + ia * (T / 2) + g);
      sp.tiles.push_back(td);
    }
    b.n_tiles = (int)sp.tiles.size() - b.tile_off;
    b.n_active = (int)sp.active.size() - b.active_off;
    part += (long long)b.n_tiles * br;
    sp.batches.push_back(b);
  }
  sp.n_partials = part;
  return sp;
}

}  // namespace hfx
