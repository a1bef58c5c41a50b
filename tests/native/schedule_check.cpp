// Host checks of the pair schedules (paper_2309_00651_amd/csrc/schedule.cpp).
//
// For every schedule built here, each pair i <= j that the kernels evaluate
// (their rule: row a, column b of a tile pair is live when b < nJ, a < nI,
// b + joff >= a inside a diagonal block, and, screened, its mask bit is set)
// is counted through the orbital order; the tests require:
//   * every pair i <= j once (unscreened), every kept pair once and no other
//     (screened), also as the union of the virtual groups of a shard split;
//   * the tile pairs of a batch touch disjoint orbitals (race-free K psi);
//   * tile pair shapes within the shape (nI <= rows, nJ <= tile, joff), slots
//     inside the batch buffer, `active` = exactly the slots with a live pair;
//   * batch offsets, tile counts and energy partials consistent;
//   * the kept kz planes of band-limited plans: compact plane index <-> kept
//     frequency one to one, for every cutoff including "keep all".
// Prints ALL OK and exits 0 when every check holds.
#include <algorithm>
#include <cstdio>
#include <numeric>
#include <random>
#include <set>
#include <vector>

#include "../../paper_2309_00651_amd/csrc/schedule.hpp"

using namespace hfx;

static long long g_checks = 0, g_fail = 0;
#define CHECK(c, ...)                                        \
  do {                                                       \
    ++g_checks;                                              \
    if (!(c)) {                                              \
      if (g_fail < 25) {                                     \
        std::printf("FAIL line %d: %s | ", __LINE__, #c);    \
        std::printf(__VA_ARGS__);                            \
        std::printf("\n");                                   \
      }                                                      \
      ++g_fail;                                              \
    }                                                        \
  } while (0)

static bool live(const TileDesc& td, int a, int b, bool masked) {
  if (a >= td.nI || b >= td.nJ) return false;
  if (td.diag && b + td.joff < a) return false;
  return !masked || keep_bit(td, a, b);
}

// Adds every evaluated pair of s to count[min * n + max]; checks the batch
// structure.
static void scan(const Schedule& s, const ScheduleShape& sh, bool masked,
                 const std::vector<int>& perm, std::vector<int>& count, const char* tag) {
  const int n = sh.n_orb, T = sh.tile, R = sh.rows;
  const int per_tile = R * (T / 2);
  long long part = 0;
  int tile_next = 0, act_next = 0;
  for (size_t k = 0; k < s.batches.size(); ++k) {
    const Batch& b = s.batches[k];
    CHECK(b.tile_off == tile_next && b.active_off == act_next, "%s batch %zu offsets", tag, k);
    CHECK(b.part_base == part, "%s batch %zu partial base", tag, k);
    CHECK(b.n_tiles >= 1 && b.n_tiles <= s.tiles_per_batch, "%s batch %zu has %d tile pairs", tag,
          k, b.n_tiles);
    std::vector<int> owner(n, -1);
    std::set<int> want;
    for (int t = b.tile_off; t < b.tile_off + b.n_tiles && t < (int)s.tiles.size(); ++t) {
      const TileDesc& td = s.tiles[t];
      CHECK(td.nI >= 1 && td.nI <= R && td.nJ >= 1 && td.nJ <= T, "%s tile %d shape %dx%d", tag,
            t, td.nI, td.nJ);
      CHECK(td.i0 >= 0 && td.i0 + td.nI <= n && td.j0 >= 0 && td.j0 + td.nJ <= n,
            "%s tile %d range", tag, t);
      CHECK(td.slot0 >= 0 && td.slot0 % per_tile == 0 && td.slot0 + per_tile <= s.slots_per_batch,
            "%s tile %d slot0 %d (budget %d)", tag, t, td.slot0, s.slots_per_batch);
      if (td.diag) {
        CHECK(td.joff == td.j0 - td.i0 && td.joff >= 0 && td.joff + td.nJ <= R, "%s tile %d joff",
              tag, t);
      } else {
        CHECK(td.joff == 0 && (td.i0 + td.nI <= td.j0 || td.j0 + td.nJ <= td.i0),
              "%s tile %d off-diagonal blocks overlap", tag, t);
      }
      if (masked) {
        for (int a = 0; a < kMaxRows; ++a)
          for (int c = 0; c < T; ++c)
            if (a >= td.nI || c >= td.nJ) CHECK(!keep_bit(td, a, c), "%s tile %d stray bit", tag, t);
      }
      // orbitals of this tile pair: rows, and columns (inside the rows when diagonal)
      std::set<int> mine;
      for (int a = 0; a < td.nI; ++a) mine.insert(td.i0 + a);
      for (int c = 0; c < td.nJ; ++c) mine.insert(td.j0 + c);
      for (int p : mine) {
        CHECK(owner[p] < 0 || owner[p] == t, "%s batch %zu: position %d in two tile pairs", tag,
              k, p);
        owner[p] = t;
      }
      for (int a = 0; a < td.nI; ++a)
        for (int c = 0; c < td.nJ; ++c) {
          if (!live(td, a, c, masked)) continue;
          const int pi = td.i0 + a, pj = td.j0 + c;
          CHECK(pi <= pj, "%s tile %d evaluates position pair %d > %d", tag, t, pi, pj);
          const int i = perm[pi], j = perm[pj];
          ++count[(size_t)std::min(i, j) * n + std::max(i, j)];
          want.insert(td.slot0 + a * (T / 2) + c / 2);
        }
    }
    std::vector<int> got(s.active.begin() + std::min<size_t>(b.active_off, s.active.size()),
                         s.active.begin() + std::min<size_t>(b.active_off + b.n_active,
                                                             s.active.size()));
    std::set<int> gset(got.begin(), got.end());
    CHECK(gset.size() == got.size(), "%s batch %zu: duplicate active slot", tag, k);
    CHECK(gset == want, "%s batch %zu: active slots %zu, live grids %zu", tag, k, gset.size(),
          want.size());
    part += (long long)b.n_tiles * sh.bricks;
    tile_next += b.n_tiles;
    act_next += b.n_active;
  }
  CHECK(tile_next == (int)s.tiles.size() && act_next == (int)s.active.size(), "%s totals", tag);
  CHECK(s.n_partials == part, "%s partials %lld vs %lld", tag, s.n_partials, part);
}

static void check_rounds() {
  for (int nb = 1; nb <= 41; ++nb) {
    const auto rounds = tile_rounds(nb);
    std::vector<int> seen(nb * nb, 0);
    for (const auto& r : rounds) {
      std::vector<int> used(nb, 0);
      for (const auto& p : r) {
        CHECK(p.first <= p.second && p.second < nb, "rounds nb=%d pair", nb);
        CHECK(!used[p.first] && (p.first == p.second || !used[p.second]), "rounds nb=%d reuse", nb);
        used[p.first] = used[p.second] = 1;
        ++seen[p.first * nb + p.second];
      }
    }
    for (int i = 0; i < nb; ++i)
      for (int j = i; j < nb; ++j) CHECK(seen[i * nb + j] == 1, "rounds nb=%d (%d,%d)", nb, i, j);
  }
}

static void check_unscreened() {
  const int sizes[] = {1, 2, 7, 8, 9, 15, 16, 17, 31, 32, 33, 37, 40, 63, 64, 65, 70, 100, 256, 257};
  for (int n : sizes)
    for (int rows : {8, 16, 24, 32})
      for (int bricks : {576, 4096})
        for (long long cap : {0LL, 1LL, 3LL})
          for (int shards : {1, 2, 3}) {
            std::vector<int> count((size_t)n * n, 0), perm(n);
            std::iota(perm.begin(), perm.end(), 0);
            char tag[96];
            for (int g = 0; g < shards; ++g) {
              ScheduleShape sh{n, 8, rows, bricks, g, shards};
              std::snprintf(tag, sizeof tag, "n=%d R=%d br=%d cap=%lld g=%d/%d", n, rows, bricks,
                            cap, g, shards);
              const Schedule s = build_schedule(sh, cap);
              CHECK(s.slots_per_batch == s.tiles_per_batch * rows * 4, "%s slots", tag);
              if (cap > 0) CHECK(s.tiles_per_batch <= cap, "%s cap", tag);
              scan(s, sh, false, perm, count, tag);
            }
            for (int i = 0; i < n; ++i)
              for (int j = i; j < n; ++j)
                CHECK(count[(size_t)i * n + j] == 1, "%s: pair (%d,%d) counted %d", tag, i, j,
                      count[(size_t)i * n + j]);
          }
}

static void check_screened() {
  std::mt19937 rng(20230901);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const int sizes[] = {1, 5, 8, 13, 37, 64, 70, 129};
  for (int n : sizes)
    for (double density : {0.0, 0.05, 0.3, 1.0})
      for (int rows : {8, 16, 32})
        for (int order = 0; order < 3; ++order)
          for (int shards : {1, 2}) {
            // symmetric overlap and kept pairs; the diagonal is kept unless nothing is
            std::vector<double> a((size_t)n * n);
            std::vector<unsigned char> keep((size_t)n * n);
            for (int i = 0; i < n; ++i)
              for (int j = i; j < n; ++j) {
                const double v = i == j ? 1.0 : u(rng);
                a[(size_t)i * n + j] = a[(size_t)j * n + i] = v;
                const unsigned char k = density > 0 && (i == j || u(rng) < density) ? 1 : 0;
                keep[(size_t)i * n + j] = keep[(size_t)j * n + i] = k;
              }
            std::vector<int> perm(n);
            std::iota(perm.begin(), perm.end(), 0);
            if (order == 1) std::shuffle(perm.begin(), perm.end(), rng);
            if (order == 2) {
              perm = cluster_order(n, 8, a, keep);
              std::vector<int> sorted(perm);
              std::sort(sorted.begin(), sorted.end());
              for (int i = 0; i < n; ++i) CHECK(sorted[i] == i, "cluster_order n=%d not a permutation", n);
            }
            // the batch buffer of the unscreened schedule
            const int slots = build_schedule(ScheduleShape{n, 8, rows, 576, 0, 1}, 0).slots_per_batch;
            std::vector<int> count((size_t)n * n, 0);
            char tag[96];
            for (int g = 0; g < shards; ++g) {
              ScheduleShape sh{n, 8, rows, 576, g, shards};
              std::snprintf(tag, sizeof tag, "screened n=%d p=%.2f R=%d order=%d g=%d/%d", n,
                            density, rows, order, g, shards);
              const Schedule s = build_screened_schedule(sh, slots, keep, perm);
              CHECK(s.slots_per_batch == slots, "%s slots", tag);
              scan(s, sh, true, perm, count, tag);
            }
            for (int i = 0; i < n; ++i)
              for (int j = i; j < n; ++j)
                CHECK(count[(size_t)i * n + j] == (int)keep[(size_t)i * n + j],
                      "%s: pair (%d,%d) counted %d, kept %d", tag, i, j, count[(size_t)i * n + j],
                      (int)keep[(size_t)i * n + j]);
          }
}

// Pruned kz planes (band-limited orbitals): the compact plane index maps
// one to one onto the kept frequencies, for every cutoff including the
// "keep all" value the plans use by default.
static void check_kz_planes() {
  for (int nz : {24, 48, 64, 72, 80, 96, 108, 120, 128})
    for (int kz_max : {0, 1, 5, nz / 2 - 1, nz / 2, nz / 2 + 1, nz, 1 << 30}) {
      if (kz_max < 0) continue;
      const int np = kz_planes(nz, kz_max);
      int kept = 0;
      for (int k = 0; k < nz; ++k) kept += kz_kept(k, nz, kz_max) ? 1 : 0;
      CHECK(np > 0 && np <= nz && np == kept, "kz nz=%d kz_max=%d planes %d kept %d", nz, kz_max,
            np, kept);
      std::vector<int> seen(nz, 0);
      for (int c = 0; c < np; ++c) {
        const int k = kz_of_plane(c, nz, kz_max);
        CHECK(k >= 0 && k < nz && kz_kept(k, nz, kz_max), "kz nz=%d kz_max=%d plane %d -> %d", nz,
              kz_max, c, k);
        if (k >= 0 && k < nz) ++seen[k];
      }
      for (int k = 0; k < nz; ++k)
        CHECK(seen[k] == (kz_kept(k, nz, kz_max) ? 1 : 0), "kz nz=%d kz_max=%d k=%d seen %d", nz,
              kz_max, k, seen[k]);
    }
}

int main() {
  check_kz_planes();
  check_rounds();
  check_unscreened();
  check_screened();
  std::printf("%lld checks, %lld failed\n", g_checks, g_fail);
  if (g_fail) return 1;
  std::printf("ALL OK\n");
  return 0;
}
