// Dense contractions over the grid: C = alpha * A B^T with A, B [n][nr]
// (orbital-major, grid points contiguous).  Used for the exchange matrix
// M = dV Psi^T (K Psi), the overlap S = dV Psi^T Psi and the float32 plans'
// pair-density means (1/N_r) Psi^T Psi.
//
// The long grid dimension is cut into chunks; one workgroup computes one
// TM x TN tile of C over one chunk on the matrix cores and stores a float64
// partial, and a second kernel sums the partials over the chunks in a fixed
// order (results are bitwise reproducible).  Inside a workgroup, K-blocks of
// KB grid points are staged through double-buffered LDS: the vector loads of
// block k+1 are in flight while block k feeds the MFMAs.  Workgroups of one
// chunk are consecutive in the XCD-aware order, so the chunk's rows of A and B
// come from HBM once and are shared through the XCD's L2.  When A and B are
// the same matrix only the tiles on and above the diagonal are computed.
//
// Split precision (float32 plans, exchange matrix): A is float64 and is split
// as a = hi + lo with hi = fl32(a), lo = fl32(a - hi); hi*b and lo*b go to two
// float32 MFMA accumulators that are folded into float64 registers every
// KFOLD grid points, so A's float64 information reaches the result and the
// float32 accumulation length stays bounded.
#include <hip/hip_runtime.h>

#include "hfx_internal.hpp"

namespace hfx {

namespace {
constexpr int KB = 16;          // grid points per LDS stage
constexpr int KFOLD = 32;       // float32 accumulation length before folding
constexpr int TARGET_WG = 512;  // workgroups per product (two per compute unit)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// MODE 0: float64 A and B, float64 MFMA.  MODE 1: split A, float32 B.
// MODE 2: as 0 on |A| and |B| (the screening overlaps int |phi_i phi_j|).
template <int MODE>
struct Cfg {
  static constexpr int TM = 128;                 // C tile rows (A rows)
  static constexpr int TN = MODE == 1 ? 64 : 128;  // C tile columns (B rows)
  static constexpr int WM = 64;                  // rows per wavefront (2 x 2 wavefronts)
  static constexpr int WN = TN / 2;
  static constexpr int BM = WM / 16, BN = WN / 16;  // 16 x 16 MFMA blocks per wavefront
};

__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// tile index -> (ti, tj); symmetric products enumerate ti <= tj row by row
__host__ __device__ inline void tile_coords(int t, int tiles_m, int tiles_n, bool sym, int& ti,
                                            int& tj) {
  if (!sym) {
    ti = t / tiles_n;
    tj = t - ti * tiles_n;
    return;
  }
  ti = 0;
  while (t >= tiles_n - ti) {
    t -= tiles_n - ti;
    ++ti;
  }
  tj = ti + t;
}

struct GemmShape {
  int tiles_m, tiles_n, n_tiles, n_chunks;
  long long chunk_len;
};

template <int MODE>
GemmShape gemm_shape(int n, long long nr, bool sym) {
  using C = Cfg<MODE>;
  GemmShape g;
  g.tiles_m = (n + C::TM - 1) / C::TM;
  g.tiles_n = (n + C::TN - 1) / C::TN;
  g.n_tiles = sym ? g.tiles_m * (g.tiles_m + 1) / 2 : g.tiles_m * g.tiles_n;
  // whole rounds: TARGET_WG workgroups run at once, one more would double
  // the time of the product
  long long chunks = TARGET_WG / g.n_tiles;
  const long long max_chunks = (nr + 4 * KB - 1) / (4 * KB);  // at least 4 K-blocks each
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  long long len = (nr + chunks - 1) / chunks;
  len = (len + KB - 1) / KB * KB;
  g.chunk_len = len;
  g.n_chunks = (int)((nr + len - 1) / len);
  return g;
}
}  // namespace

// MFMA 16x16x4 operand layout (one 64-wide wavefront, lane l):
//   A operand: A[l % 16][l / 16]   (16 x 4)
//   B operand: B[l / 16][l % 16]   (4 x 16)
//   result, 4 values i = 0..3:  f32: D[4 (l / 16) + i][l % 16]
//                               f64: D[(l / 16) + 4 i][l % 16]
// (both checked on gfx950 against a host product).
// One product of a launch: C = alpha A B^T over nr points, its chunking and
// tiles (gemm_shape), partials and output.  A launch carries up to
// kMaxGroup of them (a GramGroup, by value as the kernel argument); product s
// owns the logical workgroups [start[s], start[s + 1]) of the product kernel
// and [rstart[s], rstart[s + 1]) of the reduction.  Each product keeps its
// own chunking, so its result is the same whether launched alone or with
// others.
struct GramJob {
  const double* a;
  const void* b;
  double* part;
  double* c;
  double alpha;
  long long nr, chunk_len;
  int n, n_chunks, tiles_m, tiles_n, n_tiles, sym;
};
struct GramGroup {
  GramJob j[kMaxGroup];
  int start[kMaxGroup + 1];
  int rstart[kMaxGroup + 1];
  int count;
};
__device__ __forceinline__ int gram_locate(const int* start, int count, int L, int& s) {
  int k = 0;
#pragma unroll
  for (int i = 1; i < kMaxGroup; ++i)
    if (i < count && L >= start[i]) k = i;
  s = k;
  return L - start[k];
}

template <int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_gram(GramGroup grp) {
  int js = 0;
  const int L = gram_locate(grp.start, grp.count, xcd_order(blockIdx.x, gridDim.x), js);
  const GramJob& J = grp.j[js];
  const double* __restrict__ a = J.a;
  const void* __restrict__ bv = J.b;
  const int n = J.n, n_chunks = J.n_chunks, tiles_m = J.tiles_m, tiles_n = J.tiles_n;
  const int n_tiles = J.n_tiles, sym = J.sym;
  const long long nr = J.nr, chunk_len = J.chunk_len;
  double* __restrict__ part = J.part;
  (void)n_chunks;
  using C = Cfg<MODE>;
  constexpr int TM = C::TM, TN = C::TN, BM = C::BM, BN = C::BN;
  constexpr bool SPLIT = MODE == 1;
  using BT = typename std::conditional<SPLIT, float, double>::type;
  using AT = typename std::conditional<SPLIT, float, double>::type;  // LDS type of A
  const BT* __restrict__ b = static_cast<const BT*>(bv);
  __shared__ AT as_hi[2][TM][KB + 1];
  __shared__ float as_lo[SPLIT ? 2 : 1][SPLIT ? TM : 1][KB + 1];
  __shared__ BT bs[2][TN][KB + 1];

  const int tile = L % n_tiles, c = L / n_tiles;
  int ti, tj;
  tile_coords(tile, tiles_m, tiles_n, sym != 0, ti, tj);
  const int row0 = ti * TM, col0 = tj * TN;
  const long long r_begin = (long long)c * chunk_len;
  const long long r_end = r_begin + chunk_len < nr ? r_begin + chunk_len : nr;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * C::WM, wc = (wave & 1) * C::WN;
  const int lr = lane & 15, lk = lane >> 4;

  // loader maps: A 128 rows x 16 points (8 doubles per thread); B TN rows x
  // 16 points (8 doubles or, split, 4 floats per thread)
  const int a_row = tid >> 1, a_k = (tid & 1) * 8;
  constexpr int BPT = SPLIT ? 4 : 8;  // B values per thread
  constexpr int BTPR = KB / BPT;      // threads per B row
  const int b_row = tid / BTPR, b_k = (tid % BTPR) * BPT;
  const bool a_ok = row0 + a_row < n;
  const bool b_ok = b_row < TN && col0 + b_row < n;
  const double* __restrict__ a_ptr = a + (long long)(a_ok ? row0 + a_row : 0) * nr;
  const BT* __restrict__ b_ptr = b + (long long)(b_ok ? col0 + b_row : 0) * nr;

  double ra[8];
  BT rb[BPT];
  auto load = [&](long long r0) {
    const long long ra0 = r0 + a_k, rb0 = r0 + b_k;
    if (a_ok && ra0 + 8 <= r_end) {
      const double2* p = reinterpret_cast<const double2*>(a_ptr + ra0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 v = p[u];
        ra[2 * u] = v.x;
        ra[2 * u + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) ra[u] = (a_ok && ra0 + u < r_end) ? a_ptr[ra0 + u] : 0.0;
    }
    if constexpr (SPLIT) {
      if (b_ok && rb0 + 4 <= r_end) {
        const float4 v = *reinterpret_cast<const float4*>(b_ptr + rb0);
        rb[0] = v.x;
        rb[1] = v.y;
        rb[2] = v.z;
        rb[3] = v.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) rb[u] = (b_ok && rb0 + u < r_end) ? b_ptr[rb0 + u] : 0.f;
      }
    } else {
      if (b_ok && rb0 + 8 <= r_end) {
        const double2* p = reinterpret_cast<const double2*>(b_ptr + rb0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double2 v = p[u];
          rb[2 * u] = v.x;
          rb[2 * u + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) rb[u] = (b_ok && rb0 + u < r_end) ? b_ptr[rb0 + u] : 0.0;
      }
    }
  };
  auto stage = [&](int buf) {
    if constexpr (MODE == 2) {
#pragma unroll
      for (int u = 0; u < 8; ++u) ra[u] = fabs(ra[u]);
#pragma unroll
      for (int u = 0; u < BPT; ++u) rb[u] = fabs(rb[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if constexpr (SPLIT) {
        const float hi = (float)ra[u];
        as_hi[buf][a_row][a_k + u] = hi;
        as_lo[buf][a_row][a_k + u] = (float)(ra[u] - (double)hi);
      } else {
        as_hi[buf][a_row][a_k + u] = ra[u];
      }
    }
    if (b_row < TN) {
#pragma unroll
      for (int u = 0; u < BPT; ++u) bs[buf][b_row][b_k + u] = rb[u];
    }
  };

  f64x4 acc64[BM][BN];
  f32x4 acch[SPLIT ? BM : 1][SPLIT ? BN : 1], accl[SPLIT ? BM : 1][SPLIT ? BN : 1];
#pragma unroll
  for (int p = 0; p < BM; ++p)
#pragma unroll
    for (int q = 0; q < BN; ++q) acc64[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  if constexpr (SPLIT) {
#pragma unroll
    for (int p = 0; p < BM; ++p)
#pragma unroll
      for (int q = 0; q < BN; ++q) {
        acch[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        accl[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  }

  int buf = 0, since_fold = 0;
  if (r_begin < r_end) {
    load(r_begin);
    stage(0);
  }
  __syncthreads();
  for (long long r0 = r_begin; r0 < r_end; r0 += KB) {
    const bool more = r0 + KB < r_end;
    if (more) load(r0 + KB);  // next block in flight during the products below
#pragma unroll
    for (int s = 0; s < KB / 4; ++s) {
      const int kk = 4 * s + lk;
      if constexpr (SPLIT) {
        float ah[BM], al[BM], bx[BN];
#pragma unroll
        for (int p = 0; p < BM; ++p) {
          ah[p] = as_hi[buf][wr + 16 * p + lr][kk];
          al[p] = as_lo[buf][wr + 16 * p + lr][kk];
        }
#pragma unroll
        for (int q = 0; q < BN; ++q) bx[q] = bs[buf][wc + 16 * q + lr][kk];
#pragma unroll
        for (int p = 0; p < BM; ++p)
#pragma unroll
          for (int q = 0; q < BN; ++q) {
            acch[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[p], bx[q], acch[p][q], 0, 0, 0);
            accl[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(al[p], bx[q], accl[p][q], 0, 0, 0);
          }
      } else {
        double ad[BM], bd[BN];
#pragma unroll
        for (int p = 0; p < BM; ++p) ad[p] = as_hi[buf][wr + 16 * p + lr][kk];
#pragma unroll
        for (int q = 0; q < BN; ++q) bd[q] = bs[buf][wc + 16 * q + lr][kk];
#pragma unroll
        for (int p = 0; p < BM; ++p)
#pragma unroll
          for (int q = 0; q < BN; ++q)
            acc64[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[p], bd[q], acc64[p][q], 0, 0, 0);
      }
    }
    if constexpr (SPLIT) {
      since_fold += KB;
      if (since_fold >= KFOLD || !more) {
#pragma unroll
        for (int p = 0; p < BM; ++p)
#pragma unroll
          for (int q = 0; q < BN; ++q) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              acc64[p][q][i] += (double)acch[p][q][i] + (double)accl[p][q][i];
            acch[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
            accl[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
        since_fold = 0;
      }
    }
    if (more) stage(buf ^ 1);  // the other buffer: last read before the previous barrier
    __syncthreads();
    buf ^= 1;
  }

  double* out = part + ((long long)tile * n_chunks + c) * TM * TN;
#pragma unroll
  for (int p = 0; p < BM; ++p)
#pragma unroll
    for (int q = 0; q < BN; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = wr + 16 * p + (SPLIT ? 4 * lk + i : lk + 4 * i);
        const int cc = wc + 16 * q + lr;
        out[rr * TN + cc] = acc64[p][q][i];
      }
}

// C[i][j] = alpha * sum_c part[tile(i, j)][c][i % TM][j % TN] in a fixed
// order over c; symmetric products read (j, i) below the diagonal.
template <int MODE>
__global__ void __launch_bounds__(256) k_gram_reduce(GramGroup grp) {
  int js = 0;
  const int blk = gram_locate(grp.rstart, grp.count, (int)blockIdx.x, js);
  const GramJob& J = grp.j[js];
  const double* __restrict__ part = J.part;
  const int n = J.n, n_chunks = J.n_chunks, tiles_m = J.tiles_m, tiles_n = J.tiles_n;
  const int sym = J.sym;
  const double alpha = J.alpha;
  double* __restrict__ cmat = J.c;
  (void)tiles_m;
  using C = Cfg<MODE>;
  const long long idx = (long long)blk * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  int i = (int)(idx / n), j = (int)(idx % n);
  if (sym && i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  const int ti = i / C::TM, tj = j / C::TN;
  int tile;
  if (sym) {
    tile = 0;
    for (int r = 0; r < ti; ++r) tile += tiles_n - r;
    tile += tj - ti;
  } else {
    tile = ti * tiles_n + tj;
  }
  const double* p = part + (long long)tile * n_chunks * C::TM * C::TN +
                    (long long)(i % C::TM) * C::TN + (j % C::TN);
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += p[(long long)c * C::TM * C::TN];
  cmat[idx] = alpha * s;
}

template <int MODE>
static GramJob gram_job(const double* a, const void* b, int n, long long nr, double alpha,
                        bool sym, double* part, double* c) {
  const GemmShape g = gemm_shape<MODE>(n, nr, sym);
  GramJob j{};
  j.a = a;
  j.b = b;
  j.part = part;
  j.c = c;
  j.alpha = alpha;
  j.nr = nr;
  j.chunk_len = g.chunk_len;
  j.n = n;
  j.n_chunks = g.n_chunks;
  j.tiles_m = g.tiles_m;
  j.tiles_n = g.tiles_n;
  j.n_tiles = g.n_tiles;
  j.sym = sym ? 1 : 0;
  return j;
}

// The products of jobs[0..count) in one launch of the product kernel and
// one of the reduction.
template <int MODE>
static void launch_gram_group(const GramJob* jobs, int count, hipStream_t s) {
  GramGroup g{};
  g.count = count;
  int blocks = 0, rblocks = 0;
  for (int i = 0; i < count; ++i) {
    g.j[i] = jobs[i];
    g.start[i] = blocks;
    g.rstart[i] = rblocks;
    blocks += jobs[i].n_tiles * jobs[i].n_chunks;
    rblocks += (int)(((long long)jobs[i].n * jobs[i].n + 255) / 256);
  }
  g.start[count] = blocks;
  g.rstart[count] = rblocks;
  hipLaunchKernelGGL(k_gram<MODE>, dim3((unsigned)blocks), dim3(256), 0, s, g);
  hipLaunchKernelGGL(k_gram_reduce<MODE>, dim3((unsigned)rblocks), dim3(256), 0, s, g);
}

template <int MODE>
static void launch_gram(const double* a, const void* b, int n, long long nr, double alpha,
                        bool sym, double* part, double* c, hipStream_t s) {
  const GramJob j = gram_job<MODE>(a, b, n, nr, alpha, sym, part, c);
  launch_gram_group<MODE>(&j, 1, s);
}

size_t gemm_partial_bytes(int n_orb, long long nr) {
  size_t best = 0;
  for (int sym = 0; sym < 2; ++sym) {
    const GemmShape f = gemm_shape<0>(n_orb, nr, sym != 0);
    const size_t a = (size_t)f.n_tiles * f.n_chunks * Cfg<0>::TM * Cfg<0>::TN * 8;
    if (a > best) best = a;
  }
  const GemmShape sp = gemm_shape<1>(n_orb, nr, false);
  const size_t b = (size_t)sp.n_tiles * sp.n_chunks * Cfg<1>::TM * Cfg<1>::TN * 8;
  return b > best ? b : best;
}

void launch_xtx_split(const double* a, const float* b, int n, long long nr, double alpha,
                      double* part, double* c, hipStream_t s) {
  launch_gram<1>(a, b, n, nr, alpha, false, part, c, s);
}

void launch_xtx_f64(const double* a, const double* b, int n, long long nr, double alpha,
                    double* part, double* c, hipStream_t s) {
  launch_gram<0>(a, b, n, nr, alpha, a == b, part, c, s);
}

void launch_xtx_abs(const double* a, int n, long long nr, double alpha, double* part, double* c,
                    hipStream_t s) {
  launch_gram<2>(a, a, n, nr, alpha, true, part, c, s);
}

void launch_gram_self_group(const double* const* a, const int* n, const long long* nr,
                            const double* alpha, double* const* part, double* const* c,
                            int count, hipStream_t s) {
  GramJob jobs[kMaxGroup];
  for (int i = 0; i < count; ++i)
    jobs[i] = gram_job<0>(a[i], a[i], n[i], nr[i], alpha[i], true, part[i], c[i]);
  launch_gram_group<0>(jobs, count, s);
}

}  // namespace hfx
