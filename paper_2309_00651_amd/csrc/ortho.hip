// Loewdin orthonormalisation in float64: Psi <- S^(-1/2) Psi (orbital-major
// storage), S = dV Psi Psi^T.
//
// S^(-1/2) comes from the coupled Newton-Schulz iteration
//   Y_0 = S / c, Z_0 = I, c = max row sum of |S| (so the spectrum lies in
//   (0, 1]; c = 1 for orthonormal input, which then converges in two steps),
//   T_k = (3 I - Z_k Y_k) / 2,  Y_{k+1} = Y_k T_k,  Z_{k+1} = T_k Z_k,
// whose Z_k converges quadratically to (S/c)^(-1/2); then S^(-1/2) = Z / sqrt(c).
// Every step is three dense float64 products on the matrix cores.
// Convergence is decided on the device: the step in which max|Z Y - I| <
// 1e-10 is the last one applied, and a flag in device memory turns the
// remaining launches into no-ops, so the host never waits.
#include <hip/hip_runtime.h>

#include <cmath>

#include "hfx_internal.hpp"

namespace hfx {

namespace {
constexpr int TM = 64;
constexpr int KB = 16;
typedef double f64x4 __attribute__((ext_vector_type(4)));
}  // namespace

// C[M][N] = alpha * A[M][K] B[K][N] (row-major, leading dims lda, ldb, ldc),
// skipped entirely when *flag != 0.  4 wavefronts x (2 x 2) MFMA f64 16x16x4
// (lane l: A[l%16][l/16], B[l/16][l%16], result i = D[l/16 + 4i][l%16]).
__global__ void __launch_bounds__(256) k_gemm_nn_f64(const double* __restrict__ a, int lda,
                                                     const double* __restrict__ b, long long ldb,
                                                     double* __restrict__ c, long long ldc, int M,
                                                     long long N, int K, double alpha,
                                                     const int* __restrict__ flag) {
  if (flag && flag[0]) return;
  __shared__ double as[TM][KB + 1];
  __shared__ double bs[KB][TM + 1];
  const long long tiles_n = (N + TM - 1) / TM;
  const int ti = (int)(blockIdx.x / tiles_n);
  const long long tj = blockIdx.x % tiles_n;
  const int row0 = ti * TM;
  const long long col0 = tj * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += KB) {
    // A tile 64 x 16: 4 values per thread; B tile 16 x 64: 4 values per thread
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * 256;
      const int ar = e / KB, ak = e % KB;
      const int gr = row0 + ar, gk = k0 + ak;
      as[ar][ak] = (gr < M && gk < K) ? a[(long long)gr * lda + gk] : 0.0;
      const int bk = e / TM, bc = e % TM;
      const int gbk = k0 + bk;
      const long long gbc = col0 + bc;
      bs[bk][bc] = (gbk < K && gbc < N) ? b[(long long)gbk * ldb + gbc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[wr + p * 16 + lr][kk + lk],
                                                           bs[kk + lk][wc + q * 16 + lr],
                                                           acc[p][q], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + wr + p * 16 + lk + 4 * i;
        const long long cc = col0 + wc + q * 16 + lr;
        if (r < M && cc < N) c[(long long)r * ldc + cc] = alpha * acc[p][q][i];
      }
}

// Newton-Schulz state in device memory: st[0] done flag, st[1] completed
// steps; err: max |Z Y - I| of the current step as the bits of a
// non-negative double (ordered like the value, so an integer atomic max
// applies); scal[0] = c.
struct NsState {
  int done, steps, pad[2];
  unsigned long long err;
  double c;
};

// c = max row sum of |S| (a bound on the spectral radius of the symmetric S,
// tight when S is close to diagonal); Y0 = S / c, Z0 = I.
__global__ void __launch_bounds__(256) k_ns_init(const double* __restrict__ s, int n,
                                                 double* __restrict__ y, double* __restrict__ z,
                                                 NsState* __restrict__ st) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    double r = 0.0;
    for (int j = 0; j < n; ++j) r += fabs(s[(long long)i * n + j]);
    m = fmax(m, r);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double c = red[0];
  const long long nn = (long long)n * n;
  for (long long i = threadIdx.x; i < nn; i += 256) {
    y[i] = s[i] / c;
    z[i] = (i / n == i % n) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) {
    st->c = c;
    st->done = 0;
    st->steps = 0;
    st->err = 0ull;
  }
}

// One n x n x n float64 product C = A B on 32 x 32 tiles (4 wavefronts, one
// 16 x 16 MFMA block each), skipped once the iteration is done.  EPI: the
// first product of a step, P = Z Y, is stored as T = (3 I - P) / 2 and
// max |P - I| goes to st->err.
template <bool EPI>
__global__ void __launch_bounds__(256) k_ns_gemm(const double* __restrict__ a,
                                                 const double* __restrict__ b,
                                                 double* __restrict__ c, int n,
                                                 NsState* __restrict__ st) {
  if (st->done) return;
  constexpr int T = 32, KB = 16;
  __shared__ double as[T][KB + 1];
  __shared__ double bs[KB][T + 1];
  __shared__ double red[256];
  const int tiles = (n + T - 1) / T;
  const int row0 = (blockIdx.x / tiles) * T, col0 = (blockIdx.x % tiles) * T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 16, wc = (wave & 1) * 16;
  const int lr = lane & 15, lk = lane >> 4;
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += KB) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + 256 * u;
      const int ar = e / KB, ak = e % KB;
      as[ar][ak] = (row0 + ar < n && k0 + ak < n) ? a[(long long)(row0 + ar) * n + k0 + ak] : 0.0;
      const int bk = e / T, bc = e % T;
      bs[bk][bc] = (k0 + bk < n && col0 + bc < n) ? b[(long long)(k0 + bk) * n + col0 + bc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(as[wr + lr][kk + lk], bs[kk + lk][wc + lr], acc,
                                                 0, 0, 0);
    __syncthreads();
  }
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = row0 + wr + lk + 4 * i, cc = col0 + wc + lr;
    if (r < n && cc < n) {
      if constexpr (EPI) {
        const double d = acc[i] - (r == cc ? 1.0 : 0.0);
        m = fmax(m, fabs(d));
        c[(long long)r * n + cc] = (r == cc ? 1.0 : 0.0) - 0.5 * d;
      } else {
        c[(long long)r * n + cc] = acc[i];
      }
    }
  }
  if constexpr (EPI) {
    red[tid] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
      __syncthreads();
    }
    if (tid == 0) atomicMax(&st->err, (unsigned long long)__double_as_longlong(red[0]));
  }
}

// End of a step: count it; once max |Z Y - I| < 1e-10 the step just applied
// is the last one.
__global__ void k_ns_latch(NsState* __restrict__ st) {
  if (st->done) return;
  st->steps += 1;
  if (__longlong_as_double((long long)st->err) < 1e-10) st->done = 1;
  st->err = 0ull;
}

__global__ void __launch_bounds__(256) k_ns_final(const double* __restrict__ z0,
                                                  const double* __restrict__ z1, long long nn,
                                                  const NsState* __restrict__ st,
                                                  double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double* z = (st->steps & 1) ? z1 : z0;
  if (i < nn) out[i] = z[i] / sqrt(st->c);
}

__global__ void __launch_bounds__(256) k_copy_cols(const double* __restrict__ tmp, int n,
                                                   long long cc, double* __restrict__ psi,
                                                   long long nr, long long c0) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * cc) return;
  const long long r = i / cc, k = i % cc;
  psi[r * nr + c0 + k] = tmp[i];
}

static void gemm_nn(const double* a, int lda, const double* b, long long ldb, double* c,
                    long long ldc, int M, long long N, int K, double alpha, const int* flag,
                    hipStream_t st) {
  const long long tiles = (long long)((M + TM - 1) / TM) * ((N + TM - 1) / TM);
  hipLaunchKernelGGL(k_gemm_nn_f64, dim3((unsigned)tiles), dim3(256), 0, st, a, lda, b, ldb, c,
                     ldc, M, N, K, alpha, flag);
}

// s: n x n overlap in, S^(-1/2) out.  work: >= 5 n^2 doubles + 64 bytes.
// Step k reads (Y, Z)[k % 2] and writes (Y, Z)[(k + 1) % 2]; the final
// result is Z[steps % 2], read on the device.
hipError_t launch_inverse_sqrt(double* s, int n, double* work, int max_iter, hipStream_t st) {
  const long long nn = (long long)n * n;
  double* y[2] = {work, work + nn};
  double* z[2] = {work + 2 * nn, work + 3 * nn};
  double* t = work + 4 * nn;
  NsState* state = reinterpret_cast<NsState*>(work + 5 * nn);
  hipLaunchKernelGGL(k_ns_init, dim3(1), dim3(256), 0, st, s, n, y[0], z[0], state);
  const int tiles = (n + 31) / 32;
  const unsigned g = (unsigned)(tiles * tiles);
  for (int it = 0; it < max_iter; ++it) {
    const int cur = it & 1, nxt = cur ^ 1;
    hipLaunchKernelGGL(k_ns_gemm<true>, dim3(g), dim3(256), 0, st, z[cur], y[cur], t, n, state);
    hipLaunchKernelGGL(k_ns_gemm<false>, dim3(g), dim3(256), 0, st, y[cur], t, y[nxt], n, state);
    hipLaunchKernelGGL(k_ns_gemm<false>, dim3(g), dim3(256), 0, st, t, z[cur], z[nxt], n, state);
    hipLaunchKernelGGL(k_ns_latch, dim3(1), dim3(1), 0, st, state);
  }
  const unsigned eb = (unsigned)((nn + 255) / 256);
  hipLaunchKernelGGL(k_ns_final, dim3(eb), dim3(256), 0, st, z[0], z[1], nn, state, s);
  return hipGetLastError();
}

// psi <- m psi in place, one block of CB grid points per workgroup: the
// block (all n orbitals) is staged in LDS, so the workgroup may overwrite it
// in HBM; m (n x n, a few hundred KB) is read by every workgroup and stays in
// L2.  4 wavefronts share the output rows, BM 16-row MFMA blocks each.  The
// contraction index k is permuted per lane (lane group g = l / 16 takes
// k = k0 + 4 g + j for MFMA step j) so that each lane reads four consecutive
// m values per row with one vector load; the block rows are read from LDS in
// the same order.
// S: element type of the source (float32 sources are widened while staged).
template <int BM, int CB, typename S>
__global__ void __launch_bounds__(256) k_apply_left(const double* __restrict__ m, int n,
                                                    const S* src, double* dst, long long nr) {
  constexpr int BN = CB / 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* blk = reinterpret_cast<double*>(smem_raw);  // [k][CB + 2], k < npad
  constexpr int LD = CB + 2;                            // 16-byte aligned rows
  const int npad = (n + 15) / 16 * 16;
  const long long c0 = (long long)blockIdx.x * CB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, g = lane >> 4;
  // stage the block (rows beyond n and columns beyond nr as zeros), two
  // doubles per load: nr is even (n^3, n even) and c0 a multiple of CB
  constexpr int PR = CB / 2;  // pairs per row
  constexpr int U = 8;        // loads in flight per thread
  const int total = npad * PR;
  for (int e0 = 0; e0 < total; e0 += 256 * U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + tid + 256 * u;
      const int k = e / PR, cc = 2 * (e - k * PR);
      v[u] = double2{0.0, 0.0};
      if (e < total && k < n && c0 + cc + 1 < nr) {
        if constexpr (sizeof(S) == 8) {
          v[u] = *reinterpret_cast<const double2*>(src + (long long)k * nr + c0 + cc);
        } else {
          const float2 f = *reinterpret_cast<const float2*>(src + (long long)k * nr + c0 + cc);
          v[u] = double2{(double)f.x, (double)f.y};
        }
      } else if (e < total && k < n && c0 + cc < nr) {
        v[u].x = (double)src[(long long)k * nr + c0 + cc];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + tid + 256 * u;
      const int k = e / PR, cc = 2 * (e - k * PR);
      if (e < total) *reinterpret_cast<double2*>(blk + k * LD + cc) = v[u];
    }
  }
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  f64x4 acc[BM][BN];
#pragma unroll
  for (int p = 0; p < BM; ++p)
#pragma unroll
    for (int q = 0; q < BN; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  // m fragments of rows (wave + 4 p) * 16 + lr, k = k0 + 4 g + (0..3)
  auto load_m = [&](int k0, double (*av)[4]) {
    const int kb = k0 + 4 * g;
#pragma unroll
    for (int p = 0; p < BM; ++p) {
      const int row = (wave + 4 * p) * 16 + lr;
      if (row < n && kb + 4 <= n && (n & 1) == 0) {  // 16-byte aligned rows
        const double2* src = reinterpret_cast<const double2*>(m + (long long)row * n + kb);
        const double2 x = src[0], y = src[1];
        av[p][0] = x.x;
        av[p][1] = x.y;
        av[p][2] = y.x;
        av[p][3] = y.y;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          av[p][j] = (row < n && kb + j < n) ? m[(long long)row * n + kb + j] : 0.0;
      }
    }
  };
  double av[BM][4], an[BM][4];
  load_m(0, av);
  __syncthreads();
  for (int k0 = 0; k0 < npad; k0 += 16) {
    if (k0 + 16 < npad) load_m(k0 + 16, an);  // next fragments in flight
    const int kb = k0 + 4 * g;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double bv[BN];
#pragma unroll
      for (int q = 0; q < BN; ++q) bv[q] = blk[(kb + j) * LD + 16 * q + lr];
#pragma unroll
      for (int p = 0; p < BM; ++p)
#pragma unroll
        for (int q = 0; q < BN; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p][j], bv[q], acc[p][q], 0, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < BM; ++p)
#pragma unroll
      for (int j = 0; j < 4; ++j) av[p][j] = an[p][j];
  }
  // result i of lane l: row (l / 16) + 4 i of the block, column l % 16
#pragma unroll
  for (int p = 0; p < BM; ++p)
#pragma unroll
    for (int q = 0; q < BN; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = (wave + 4 * p) * 16 + g + 4 * i;
        const long long col = c0 + 16 * q + lr;
        if (row < n && col < nr) dst[(long long)row * nr + col] = acc[p][q][i];
      }
}

// dst <- m src (n x n times n x nr; dst == src allowed: each workgroup reads
// its whole column block before writing it).  n <= 512: one pass
// (k_apply_left); larger n: column chunks through tmp (n x 32768 doubles)
// and a copy to dst.
void launch_apply_left(const double* m, const double* src, double* dst, int n, long long nr,
                       double* tmp, hipStream_t st) {
  if (n <= 256) {
    constexpr int CB = 32;
    const size_t lds = (size_t)((n + 15) / 16 * 16) * (CB + 2) * 8;
    hipLaunchKernelGGL((k_apply_left<4, CB, double>), dim3((unsigned)((nr + CB - 1) / CB)), dim3(256),
                       lds, st, m, n, src, dst, nr);
    return;
  }
  if (n <= 512) {
    constexpr int CB = 16;
    const size_t lds = (size_t)((n + 15) / 16 * 16) * (CB + 2) * 8;
    hipLaunchKernelGGL((k_apply_left<8, CB, double>), dim3((unsigned)((nr + CB - 1) / CB)), dim3(256),
                       lds, st, m, n, src, dst, nr);
    return;
  }
  const long long cc = 32768;
  for (long long c0 = 0; c0 < nr; c0 += cc) {
    const long long w = c0 + cc <= nr ? cc : nr - c0;
    gemm_nn(m, n, src + c0, nr, tmp, w, n, w, n, 1.0, nullptr, st);
    const long long tot = (long long)n * w;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, tmp,
                       n, w, dst, nr, c0);
  }
}

// dst <- m widen(src) for a float32 source (n <= 512, dst distinct from
// src); returns false for larger n, where the caller widens first.
bool launch_apply_left_f32(const double* m, const float* src, double* dst, int n, long long nr,
                           hipStream_t st) {
  if (n <= 256) {
    constexpr int CB = 32;
    const size_t lds = (size_t)((n + 15) / 16 * 16) * (CB + 2) * 8;
    hipLaunchKernelGGL((k_apply_left<4, CB, float>), dim3((unsigned)((nr + CB - 1) / CB)),
                       dim3(256), lds, st, m, n, src, dst, nr);
    return true;
  }
  if (n <= 512) {
    constexpr int CB = 16;
    const size_t lds = (size_t)((n + 15) / 16 * 16) * (CB + 2) * 8;
    hipLaunchKernelGGL((k_apply_left<8, CB, float>), dim3((unsigned)((nr + CB - 1) / CB)),
                       dim3(256), lds, st, m, n, src, dst, nr);
    return true;
  }
  return false;
}

// Raise the dynamic-LDS limit of the in-place kernels (once per process).
hipError_t prepare_apply_left() {
  const void* k[4] = {reinterpret_cast<const void*>(&k_apply_left<4, 32, double>),
                      reinterpret_cast<const void*>(&k_apply_left<8, 16, double>),
                      reinterpret_cast<const void*>(&k_apply_left<4, 32, float>),
                      reinterpret_cast<const void*>(&k_apply_left<8, 16, float>)};
  const int bytes[4] = {256 * 34 * 8, 512 * 18 * 8, 256 * 34 * 8, 512 * 18 * 8};
  for (int i = 0; i < 4; ++i) {
    hipError_t e = hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize, bytes[i]);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hfx
