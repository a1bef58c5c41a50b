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

#include <cmath>

#include "hfx_internal.hpp"

namespace hfx {

namespace {
constexpr int NT = 1024;
}

// l <- lower Cholesky factor of sign * m (n x n, row-major, upper part
// zeroed).  A pivot that is not positive (sign * m not positive definite:
// dependent or zero orbitals) is stored as NaN, so everything built from L is
// NaN.
__global__ void __launch_bounds__(NT) k_chol(const double* __restrict__ m, int n, double sign,
                                             double* __restrict__ l) {
  const int tid = threadIdx.x;
  const long long nn = (long long)n * n;
  for (long long e = tid; e < nn; e += NT) {
    const int i = (int)(e / n), k = (int)(e - (long long)i * n);
    l[e] = k <= i ? sign * m[e] : 0.0;
  }
  __shared__ double piv;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = l[(long long)j * n + j];
      piv = d > 0.0 ? sqrt(d) : NAN;
      l[(long long)j * n + j] = piv;
    }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int i = j + 1 + tid; i < n; i += NT) l[(long long)i * n + j] *= inv;
    __syncthreads();
    // trailing update of the lower triangle: l[i][k] -= l[i][j] l[k][j], j < k <= i
    const int r = n - j - 1;  // trailing order
    const long long cnt = (long long)r * (r + 1) / 2;
    for (long long e = tid; e < cnt; e += NT) {
      // e -> (a, b), 0 <= b <= a < r, row-major over the triangle
      int a = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while ((long long)a * (a + 1) / 2 > e) --a;
      while ((long long)(a + 1) * (a + 2) / 2 <= e) ++a;
      const int b = (int)(e - (long long)a * (a + 1) / 2);
      const int i = j + 1 + a, k = j + 1 + b;
      l[(long long)i * n + k] -= l[(long long)i * n + j] * l[(long long)k * n + j];
    }
    __syncthreads();
  }
}

// x <- l^(-1) for lower triangular l (n x n, row-major): row i of X is
// (e_i - sum_{k<i} l[i][k] X[k]) / l[i][i], the rows before i being final.
// Each column j is summed by NT / n threads (fixed split, fixed order).
__global__ void __launch_bounds__(NT) k_trinv(const double* __restrict__ l, int n,
                                              double* __restrict__ x) {
  const int tid = threadIdx.x;
  const int parts = n >= NT ? 1 : NT / n;  // threads per column
  __shared__ double red[NT];
  for (int i = 0; i < n; ++i) {
    const double li = l[(long long)i * n + i];
    for (int c0 = 0; c0 < n; c0 += NT / parts) {
      const int j = c0 + tid % (NT / parts), part = tid / (NT / parts);
      double s = 0.0;
      if (j < n && part < parts) {
        // only k >= j contribute (X is lower triangular)
        for (int k = j + part; k < i; k += parts) s += l[(long long)i * n + k] * x[(long long)k * n + j];
      }
      red[tid] = s;
      __syncthreads();
      if (part == 0 && j < n) {
        double t = 0.0;
        for (int q = 0; q < parts; ++q) t += red[tid + q * (NT / parts)];
        x[(long long)i * n + j] = j > i ? 0.0 : ((i == j ? 1.0 : 0.0) - t) / li;
      }
      __syncthreads();
    }
  }
}

void launch_chol(const double* m, int n, double sign, double* l, hipStream_t s) {
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(NT), 0, s, m, n, sign, l);
}

void launch_trinv(const double* l, int n, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_trinv, dim3(1), dim3(NT), 0, s, l, n, x);
}

}  // namespace hfx
