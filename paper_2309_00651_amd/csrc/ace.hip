// Adaptively compressed exchange (ACE), Eq. (vx_ace) in the Methods' MTACE
// subsection: V_X^ACE = - sum_k |P_k><P_k| with P = W L^(-T), W_i = V_X psi_i
// and -M = L L^T (Cholesky).  Rows of P are the rows of L^(-1) W.  The same
// factorisation and inverse give the Cholesky orthonormalisation
// Psi <- L^(-1) Psi with S = L L^T.
//
// The n x n factorisation and the triangular inverse are small (n = N_orb)
// and run in one workgroup each on the L2-resident matrix; the grid-sized
// products (P = L^(-1) W, and the application -P (P^T phi)) use the MFMA
// contraction and in-place apply kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "hfx_internal.hpp"

namespace hfx {

namespace {
constexpr int CB = 32;   // block order of the blocked factorisation and inverse
constexpr int CT = 256;  // threads per workgroup
}

// l[i][k] = sign * m[i][k] for k <= i, 0 above the diagonal.
__global__ void __launch_bounds__(CT) k_chol_init(const double* __restrict__ m, int n,
                                                  double sign, double* __restrict__ l) {
  const long long nn = (long long)n * n;
  for (long long e = (long long)blockIdx.x * CT + threadIdx.x; e < nn;
       e += (long long)gridDim.x * CT) {
    const int i = (int)(e / n), k = (int)(e - (long long)i * n);
    l[e] = k <= i ? sign * m[e] : 0.0;
  }
}

// Inverse of the lower triangular b x b block la (b <= CB, zero-padded to
// CB): column c of the inverse solves la y = e_c by forward substitution, one
// column per thread of the first CB threads.  Entries outside b x b are 0.
__device__ __forceinline__ void block_inverse(const double (*la)[CB + 1], int b,
                                              double (*dinv)[CB + 1], int tid) {
  if (tid < CB) {
    const int c = tid;
    double y[CB];
#pragma unroll
    for (int r = 0; r < CB; ++r) {
      double s = r == c ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < r; ++q) s -= la[r][q] * y[q];
      y[r] = (r < b && r >= c) ? s / la[r][r] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < CB; ++r) dinv[r][c] = y[r];
  }
}

// Right-looking blocked Cholesky, block column at k0: factor the diagonal
// block L_kk in LDS (unblocked, column by column), invert it, and form the
// rows below, L_ik = A_ik L_kk^(-T), eight rows at a time with one output
// per thread.  A pivot that is not positive is stored as NaN, so everything
// built from L is NaN.
__global__ void __launch_bounds__(CT) k_chol_panel(double* __restrict__ l, int n, int k0) {
  __shared__ double d[CB][CB + 1], dinv[CB][CB + 1], rows[CT / CB][CB + 1];
  const int tid = threadIdx.x;
  const int b = min(CB, n - k0);
  for (int e = tid; e < CB * CB; e += CT) {
    const int r = e / CB, c = e - r * CB;
    d[r][c] = (r < b && c <= r) ? l[(long long)(k0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    const double p = d[j][j];
    const double piv = p > 0.0 ? sqrt(p) : NAN;
    __syncthreads();  // every thread has read d[j][j]
    if (tid == 0) d[j][j] = piv;
    const double inv = 1.0 / piv;
    for (int r = j + 1 + tid; r < b; r += CT) d[r][j] *= inv;
    __syncthreads();
    const int t = b - j - 1;
    for (int e = tid; e < t * t; e += CT) {
      const int r = j + 1 + e / t, c = j + 1 + e % t;
      if (c <= r) d[r][c] -= d[r][j] * d[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < CB * CB; e += CT) {
    const int r = e / CB, c = e - r * CB;
    if (r < b && c <= r) l[(long long)(k0 + r) * n + k0 + c] = d[r][c];
  }
  if (k0 + b >= n) return;  // last block column: no rows below
  block_inverse(d, b, dinv, tid);  // b == CB here
  constexpr int RPI = CT / CB;     // rows per iteration
  const int rr = tid / CB, c = tid - rr * CB;
  for (int row0 = k0 + CB; row0 < n; row0 += RPI) {
    __syncthreads();  // dinv ready; previous rows consumed
    const int row = row0 + rr;
    rows[rr][c] = row < n ? l[(long long)row * n + k0 + c] : 0.0;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q <= c; ++q) s += rows[rr][q] * dinv[c][q];
    if (row < n) l[(long long)row * n + k0 + c] = s;
  }
}

// Trailing update after the block column at k0 (a full block, k0 + CB < n):
// l[i][j] -= sum_c l[i][k0 + c] l[j][k0 + c] for i >= j >= k0 + CB, one
// workgroup per 32 x 32 tile (ti, tj), ti >= tj, of the trailing triangle.
__global__ void __launch_bounds__(CT) k_chol_update(double* __restrict__ l, int n, int k0) {
  __shared__ double pa[CB][CB + 1], pb[CB][CB + 1];
  const int k1 = k0 + CB;
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tid = threadIdx.x;
  const int i0 = k1 + ti * CB, j0 = k1 + t * CB;
  for (int e = tid; e < CB * CB; e += CT) {
    const int r = e / CB, c = e - r * CB;
    pa[r][c] = i0 + r < n ? l[(long long)(i0 + r) * n + k0 + c] : 0.0;
    pb[r][c] = j0 + r < n ? l[(long long)(j0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < CB * CB; e += CT) {
    const int r = e / CB, c = e - r * CB;
    const int i = i0 + r, j = j0 + c;
    if (i < n && j <= i) {
      double s = 0.0;
#pragma unroll 8
      for (int q = 0; q < CB; ++q) s += pa[r][q] * pb[c][q];
      l[(long long)i * n + j] -= s;
    }
  }
}

// Block row ib of X = L^(-1) (L lower triangular, n x n row-major), the rows
// above being final: workgroup kb < ib forms
// X_(ib,kb) = -X_(ib,ib) sum_(jb = kb .. ib-1) L_(ib,jb) X_(jb,kb); workgroup
// ib writes X_(ib,ib), the inverse of the diagonal block (recomputed by
// every workgroup that needs it); blocks kb > ib are zero.
__global__ void __launch_bounds__(CT) k_trinv_row(const double* __restrict__ l, int n, int ib,
                                                  double* __restrict__ x) {
  __shared__ double dinv[CB][CB + 1], la[CB][CB + 1], xb[CB][CB + 1];
  const int kb = blockIdx.x, tid = threadIdx.x;
  const int i0 = ib * CB, bi = min(CB, n - i0);
  const int c0 = kb * CB, bc = min(CB, n - c0);
  if (kb > ib) {
    for (int e = tid; e < CB * CB; e += CT) {
      const int r = e / CB, c = e - r * CB;
      if (r < bi && c < bc) x[(long long)(i0 + r) * n + c0 + c] = 0.0;
    }
    return;
  }
  for (int e = tid; e < CB * CB; e += CT) {
    const int r = e / CB, c = e - r * CB;
    la[r][c] = (r < bi && c <= r) ? l[(long long)(i0 + r) * n + i0 + c] : 0.0;
  }
  __syncthreads();
  block_inverse(la, bi, dinv, tid);
  __syncthreads();
  if (kb == ib) {
    for (int e = tid; e < CB * CB; e += CT) {
      const int r = e / CB, c = e - r * CB;
      if (r < bi && c < bi) x[(long long)(i0 + r) * n + i0 + c] = dinv[r][c];
    }
    return;
  }
  // this thread's outputs: (r, c) = (e / CB, e % CB) for e = tid + k CT
  constexpr int PER = CB * CB / CT;
  double acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0;
  for (int jb = kb; jb < ib; ++jb) {
    __syncthreads();
    for (int e = tid; e < CB * CB; e += CT) {
      const int r = e / CB, c = e - r * CB;
      la[r][c] = r < bi ? l[(long long)(i0 + r) * n + jb * CB + c] : 0.0;
      xb[r][c] = x[(long long)(jb * CB + r) * n + c0 + c];  // jb < ib: full block rows
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * CT, r = e / CB, c = e - r * CB;
      double s = acc[k];
#pragma unroll 8
      for (int q = 0; q < CB; ++q) s += la[r][q] * xb[q][c];
      acc[k] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * CT, r = e / CB, c = e - r * CB;
    xb[r][c] = acc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * CT, r = e / CB, c = e - r * CB;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < CB; ++q) s += dinv[r][q] * xb[q][c];
    if (r < bi) x[(long long)(i0 + r) * n + c0 + c] = -s;
  }
}

void launch_chol(const double* m, int n, double sign, double* l, hipStream_t s) {
  const long long nn = (long long)n * n;
  const int g = (int)std::min<long long>((nn + CT - 1) / CT, 4096);
  hipLaunchKernelGGL(k_chol_init, dim3(g), dim3(CT), 0, s, m, n, sign, l);
  for (int k0 = 0; k0 < n; k0 += CB) {
    hipLaunchKernelGGL(k_chol_panel, dim3(1), dim3(CT), 0, s, l, n, k0);
    if (k0 + CB < n) {
      const int nt = (n - k0 - CB + CB - 1) / CB;
      hipLaunchKernelGGL(k_chol_update, dim3(nt * (nt + 1) / 2), dim3(CT), 0, s, l, n, k0);
    }
  }
}

void launch_trinv(const double* l, int n, double* x, hipStream_t s) {
  const int nb = (n + CB - 1) / CB;
  for (int ib = 0; ib < nb; ++ib)
    hipLaunchKernelGGL(k_trinv_row, dim3(nb), dim3(CT), 0, s, l, n, ib, x);
}

}  // namespace hfx
