// Loewdin orthonormalisation in float64: Psi <- S^(-1/2) Psi (orbital-major
// storage), S = dV Psi Psi^T.
//
// S^(-1/2) comes from the coupled Newton-Schulz iteration
//   Y_0 = S / c, Z_0 = I, c = ||S||_F (so the spectrum lies in (0, 1]),
//   T_k = (3 I - Z_k Y_k) / 2,  Y_{k+1} = Y_k T_k,  Z_{k+1} = T_k Z_k,
// whose Z_k converges quadratically to (S/c)^(-1/2); then S^(-1/2) = Z / sqrt(c).
// Every step is a dense float64 product on the matrix cores.  Convergence is
// decided on the device: once max|Z Y - I| < 1e-10 one more step is applied
// and a flag in device memory turns the remaining launches into no-ops, so
// the host never waits.
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

// state: [0] done flag, [1] converge-after-this-step flag; scal: [0] = c
__global__ void __launch_bounds__(256) k_ns_init(const double* __restrict__ s, int n,
                                                 double* __restrict__ y, double* __restrict__ z,
                                                 int* __restrict__ state,
                                                 double* __restrict__ scal) {
  __shared__ double red[256];
  double acc = 0.0;
  const long long nn = (long long)n * n;
  for (long long i = threadIdx.x; i < nn; i += 256) acc += s[i] * s[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double c = sqrt(red[0]);
  for (long long i = threadIdx.x; i < nn; i += 256) {
    y[i] = s[i] / c;
    z[i] = (i / n == i % n) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) {
    scal[0] = c;
    state[0] = 0;
    state[1] = 0;
  }
}

// t = (3 I - p) / 2 and convergence test on max|p - I| (one workgroup).
__global__ void __launch_bounds__(256) k_ns_tform(const double* __restrict__ p, int n,
                                                  double* __restrict__ t,
                                                  int* __restrict__ state) {
  if (state[0]) return;
  __shared__ double red[256];
  double m = 0.0;
  const long long nn = (long long)n * n;
  for (long long i = threadIdx.x; i < nn; i += 256) {
    const double id = (i / n == i % n) ? 1.0 : 0.0;
    const double d = p[i] - id;
    m = fmax(m, fabs(d));
    t[i] = id - 0.5 * d;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] < 1e-10) state[1] = 1;
}

// y <- y2, z <- z2; latch the done flag after a converged step.
__global__ void __launch_bounds__(256) k_ns_commit(double* __restrict__ y,
                                                   const double* __restrict__ y2,
                                                   double* __restrict__ z,
                                                   const double* __restrict__ z2, long long nn,
                                                   int* __restrict__ state) {
  if (state[0]) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) {
    y[i] = y2[i];
    z[i] = z2[i];
  }
}

__global__ void k_ns_latch(int* __restrict__ state) {
  if (state[1]) state[0] = 1;
}

__global__ void __launch_bounds__(256) k_ns_final(const double* __restrict__ z, long long nn,
                                                  const double* __restrict__ scal,
                                                  double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) out[i] = z[i] / sqrt(scal[0]);
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
hipError_t launch_inverse_sqrt(double* s, int n, double* work, int max_iter, hipStream_t st) {
  const long long nn = (long long)n * n;
  double* y = work;
  double* z = y + nn;
  double* p = z + nn;
  double* y2 = p + nn;
  double* z2 = y2 + nn;
  int* state = reinterpret_cast<int*>(z2 + nn);
  double* scal = reinterpret_cast<double*>(state + 4);
  hipLaunchKernelGGL(k_ns_init, dim3(1), dim3(256), 0, st, s, n, y, z, state, scal);
  const unsigned eb = (unsigned)((nn + 255) / 256);
  for (int it = 0; it < max_iter; ++it) {
    gemm_nn(z, n, y, n, p, n, n, n, n, 1.0, state, st);                // p = Z Y
    hipLaunchKernelGGL(k_ns_tform, dim3(1), dim3(256), 0, st, p, n, p, state);  // p <- T
    gemm_nn(y, n, p, n, y2, n, n, n, n, 1.0, state, st);               // Y T
    gemm_nn(p, n, z, n, z2, n, n, n, n, 1.0, state, st);               // T Z
    hipLaunchKernelGGL(k_ns_commit, dim3(eb), dim3(256), 0, st, y, y2, z, z2, nn, state);
    hipLaunchKernelGGL(k_ns_latch, dim3(1), dim3(1), 0, st, state);
  }
  hipLaunchKernelGGL(k_ns_final, dim3(eb), dim3(256), 0, st, z, nn, scal, s);
  return hipGetLastError();
}

// psi <- m psi in column chunks through tmp (n x chunk doubles).
void launch_apply_left(const double* m, double* psi, int n, long long nr, double* tmp,
                       hipStream_t st) {
  const long long cc = 32768;
  for (long long c0 = 0; c0 < nr; c0 += cc) {
    const long long w = c0 + cc <= nr ? cc : nr - c0;
    gemm_nn(m, n, psi + c0, nr, tmp, w, n, w, n, 1.0, nullptr, st);
    const long long tot = (long long)n * w;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, tmp,
                       n, w, psi, nr, c0);
  }
}

}  // namespace hfx
