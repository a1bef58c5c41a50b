// Dense contractions over the grid: C = alpha * A B^T with A, B [n][nr]
// (orbital-major, grid points contiguous).  Used for the ACE matrix
// M = dV Psi^T (K Psi) and the overlap S = dV Psi^T Psi.
//
// The long grid dimension is split into chunks; each workgroup computes a
// 64 x 64 tile of C over one chunk on the matrix cores (4 wavefronts, each a
// 32 x 32 sub-tile of 2 x 2 MFMA 16x16x4 blocks) and stores a float64
// partial; a second kernel sums the partials over chunks in a fixed order.
//
// Split precision (float32 plans): A is float64 and is split as
// a = hi + lo with hi = fl32(a), lo = fl32(a - hi); hi*b and lo*b go to two
// float32 MFMA accumulators that are folded into float64 registers every
// KFOLD grid points, so A's float64 information reaches the result and the
// float32 accumulation length stays bounded.
#include <hip/hip_runtime.h>

#include "hfx_internal.hpp"

namespace hfx {

namespace {
constexpr int TM = 64;        // C tile
constexpr int KB = 32;        // grid points per LDS stage
constexpr int KFOLD = 32;     // float32 accumulation length before folding
constexpr int PAD = 1;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
}  // namespace

// MFMA 16x16x4 operand layout (one 64-wide wavefront, lane l):
//   A operand: A[l % 16][l / 16]   (16 x 4)
//   B operand: B[l / 16][l % 16]   (4 x 16)
//   result, 4 values i = 0..3:  f32: D[4 (l / 16) + i][l % 16]
//                               f64: D[(l / 16) + 4 i][l % 16]
// (both checked on gfx950 against a host product).
template <bool SPLIT>
__global__ void __launch_bounds__(256) k_xtx(const double* __restrict__ a,
                                             const void* __restrict__ bv, int n, long long nr,
                                             long long chunk_len, int n_chunks,
                                             double* __restrict__ part) {
  using BT = typename std::conditional<SPLIT, float, double>::type;
  const BT* __restrict__ b = static_cast<const BT*>(bv);
  __shared__ float ahi_s[SPLIT ? TM : 1][KB + PAD];
  __shared__ float alo_s[SPLIT ? TM : 1][KB + PAD];
  __shared__ float bf_s[SPLIT ? TM : 1][KB + PAD];
  __shared__ double ad_s[SPLIT ? 1 : TM][KB + PAD];
  __shared__ double bd_s[SPLIT ? 1 : TM][KB + PAD];

  const int tiles = (n + TM - 1) / TM;
  const int c = blockIdx.x % n_chunks;
  const int tile = blockIdx.x / n_chunks;
  const int ti = tile / tiles, tj = tile % tiles;
  const int row0 = ti * TM, col0 = tj * TM;
  const long long r_begin = (long long)c * chunk_len;
  long long r_end = r_begin + chunk_len;
  if (r_end > nr) r_end = nr;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  double accd[2][2][4];
  f32x4 acch[2][2], accl[2][2];
  f64x4 acc64[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int i = 0; i < 4; ++i) accd[p][q][i] = 0.0;
      acch[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
      accl[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc64[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
    }

  // loader mapping: 256 threads, 64 rows x 32 points -> 8 points per thread
  const int ld_row = tid >> 2, ld_k = (tid & 3) * 8;
  int since_fold = 0;
  for (long long r0 = r_begin; r0 < r_end; r0 += KB) {
    {
      const int ga = row0 + ld_row, gb = col0 + ld_row;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const long long r = r0 + ld_k + u;
        const bool rin = r < r_end;
        const double av = (ga < n && rin) ? a[(long long)ga * nr + r] : 0.0;
        const BT bvv = (gb < n && rin) ? b[(long long)gb * nr + r] : BT(0);
        if constexpr (SPLIT) {
          const float hi = (float)av;
          ahi_s[ld_row][ld_k + u] = hi;
          alo_s[ld_row][ld_k + u] = (float)(av - (double)hi);
          bf_s[ld_row][ld_k + u] = bvv;
        } else {
          ad_s[ld_row][ld_k + u] = av;
          bd_s[ld_row][ld_k + u] = bvv;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int ar = wr + p * 16 + lr, bc = wc + q * 16 + lr;
          if constexpr (SPLIT) {
            const float bx = bf_s[bc][kk + lk];
            acch[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ahi_s[ar][kk + lk], bx, acch[p][q],
                                                              0, 0, 0);
            accl[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(alo_s[ar][kk + lk], bx, accl[p][q],
                                                              0, 0, 0);
          } else {
            acc64[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad_s[ar][kk + lk],
                                                               bd_s[bc][kk + lk], acc64[p][q], 0,
                                                               0, 0);
          }
        }
    }
    __syncthreads();
    if constexpr (SPLIT) {
      since_fold += KB;
      if (since_fold >= KFOLD || r0 + KB >= r_end) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              accd[p][q][i] += (double)acch[p][q][i] + (double)accl[p][q][i];
            acch[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
            accl[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
        since_fold = 0;
      }
    }
  }
  double* out = part + ((long long)tile * n_chunks + c) * TM * TM;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = wr + p * 16 + (SPLIT ? 4 * lk + i : lk + 4 * i);
        const int cc = wc + q * 16 + lr;
        out[rr * TM + cc] = SPLIT ? accd[p][q][i] : acc64[p][q][i];
      }
}

// C[i][j] = alpha * sum_c part[tile(i,j)][c][i%64][j%64], fixed order in c.
__global__ void __launch_bounds__(256) k_xtx_reduce(const double* __restrict__ part, int n,
                                                    int n_chunks, double alpha,
                                                    double* __restrict__ cmat) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const int tiles = (n + TM - 1) / TM;
  const int tile = (i / TM) * tiles + (j / TM);
  const double* p = part + (long long)tile * n_chunks * TM * TM + (i % TM) * TM + (j % TM);
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += p[(long long)c * TM * TM];
  cmat[idx] = alpha * s;
}

int gemm_chunks(int n_orb, long long nr) {
  const int tiles = (n_orb + TM - 1) / TM;
  long long chunks = (2048 + tiles * tiles - 1) / (tiles * tiles);
  const long long max_chunks = (nr + 4 * KFOLD - 1) / (4 * KFOLD);
  if (chunks > max_chunks) chunks = max_chunks;
  if (chunks < 1) chunks = 1;
  return (int)chunks;
}

static void launch_xtx(bool split, const double* a, const void* b, int n, long long nr,
                       double alpha, double* part, int n_chunks, double* c, hipStream_t s) {
  const int tiles = (n + TM - 1) / TM;
  long long chunk_len = (nr + n_chunks - 1) / n_chunks;
  chunk_len = (chunk_len + KB - 1) / KB * KB;
  const int blocks = tiles * tiles * n_chunks;
  if (split)
    hipLaunchKernelGGL(k_xtx<true>, dim3(blocks), dim3(256), 0, s, a, b, n, nr, chunk_len,
                       n_chunks, part);
  else
    hipLaunchKernelGGL(k_xtx<false>, dim3(blocks), dim3(256), 0, s, a, b, n, nr, chunk_len,
                       n_chunks, part);
  const long long total = (long long)n * n;
  hipLaunchKernelGGL(k_xtx_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, part,
                     n, n_chunks, alpha, c);
}

void launch_xtx_split(const double* a, const float* b, int n, long long nr, double alpha,
                      double* part, int n_chunks, double* c, hipStream_t s) {
  launch_xtx(true, a, b, n, nr, alpha, part, n_chunks, c, s);
}

void launch_xtx_f64(const double* a, const double* b, int n, long long nr, double alpha,
                    double* part, int n_chunks, double* c, hipStream_t s) {
  launch_xtx(false, a, b, n, nr, alpha, part, n_chunks, c, s);
}

}  // namespace hfx
