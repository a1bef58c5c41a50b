// SCDM localisation (selected columns of the density matrix; the Methods'
// MTACE subsection uses SCDM-localised orbitals for s-MTACE).  Grid points
// c_1..c_N are chosen by column-pivoted QR of the N_orb x N_r matrix Psi^T:
// step k takes the point whose residual, after the directions of the points
// chosen so far are projected out, has the largest norm (ties: the smallest
// index).  The localised functions xi_k(r) = sum_i psi_i(r) psi_i(c_k) are the
// density-matrix columns at those points; the caller orthonormalises them.
//
// Only the pivots are needed, so no Q or R of the N_r columns is formed: the
// squared residual norms w_r are kept and downdated, w_r -= (q_k . a_r)^2,
// after each step, where q_k (N_orb values) is the normalised residual of the
// chosen column, obtained by classical Gram-Schmidt applied twice against
// q_1..q_(k-1) in one workgroup.  Each step reads Psi once (grid-wide pass)
// and runs one single-workgroup pick; the argmax is reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "hfx_internal.hpp"

namespace hfx {

namespace {
constexpr int NTS = 256;  // threads per workgroup
}

// (v, i) wins over (u, j): larger value, then smaller index
__device__ __forceinline__ bool beats(double v, long long i, double u, long long j) {
  return v > u || (v == u && i < j);
}

__device__ void block_argmax(double& v, long long& i, double* sv, long long* si) {
  const int tid = threadIdx.x;
  sv[tid] = v;
  si[tid] = i;
  __syncthreads();
  for (int s = NTS / 2; s > 0; s >>= 1) {
    if (tid < s && beats(sv[tid + s], si[tid + s], sv[tid], si[tid])) {
      sv[tid] = sv[tid + s];
      si[tid] = si[tid + s];
    }
    __syncthreads();
  }
  v = sv[0];
  i = si[0];
  __syncthreads();
}

// w_r = sum_i psi_i(r)^2, and the argmax of w over this workgroup's points
__global__ void __launch_bounds__(NTS) k_scdm_norms(const double* __restrict__ psi, int n,
                                                     long long nr, double* __restrict__ w,
                                                     double* __restrict__ pv,
                                                     long long* __restrict__ pi) {
  __shared__ double sv[NTS];
  __shared__ long long si[NTS];
  double best = -1.0;
  long long bi = LLONG_MAX;
  for (long long r = (long long)blockIdx.x * NTS + threadIdx.x; r < nr;
       r += (long long)gridDim.x * NTS) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double x = psi[(long long)i * nr + r];
      s += x * x;
    }
    w[r] = s;
    if (beats(s, r, best, bi)) {
      best = s;
      bi = r;
    }
  }
  block_argmax(best, bi, sv, si);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = best;
    pi[blockIdx.x] = bi;
  }
}

// w_r -= (q . a_r)^2 for the points not chosen yet (chosen points hold -1),
// and the argmax of the new w over this workgroup's points
__global__ void __launch_bounds__(NTS) k_scdm_update(const double* __restrict__ psi, int n,
                                                      long long nr, const double* __restrict__ q,
                                                      double* __restrict__ w,
                                                      double* __restrict__ pv,
                                                      long long* __restrict__ pi) {
  extern __shared__ double qs[];  // n values
  __shared__ double sv[NTS];
  __shared__ long long si[NTS];
  for (int i = threadIdx.x; i < n; i += NTS) qs[i] = q[i];
  __syncthreads();
  double best = -1.0;
  long long bi = LLONG_MAX;
  for (long long r = (long long)blockIdx.x * NTS + threadIdx.x; r < nr;
       r += (long long)gridDim.x * NTS) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += qs[i] * psi[(long long)i * nr + r];
    double v = w[r];
    if (v >= 0.0) {
      v = fmax(v - t * t, 0.0);
      w[r] = v;
    }
    if (beats(v, r, best, bi)) {
      best = v;
      bi = r;
    }
  }
  block_argmax(best, bi, sv, si);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = best;
    pi[blockIdx.x] = bi;
  }
}

// Step k: the global argmax of the per-workgroup candidates is the pivot;
// its column a = (psi_i(c_k))_i is orthogonalised against q_0..q_(k-1)
// (rows of qm) twice and normalised into q_k.  A vanishing residual (linearly
// dependent orbitals) gives NaN, which every later result inherits.
__global__ void __launch_bounds__(NTS) k_scdm_pick(const double* __restrict__ pv,
                                                    const long long* __restrict__ pi, int nparts,
                                                    const double* __restrict__ psi, int n,
                                                    long long nr, int k, double* __restrict__ qm,
                                                    int* __restrict__ piv,
                                                    double* __restrict__ w) {
  extern __shared__ double sh[];  // a[n], c[n]
  double* a = sh;
  double* c = sh + n;
  __shared__ double sv[NTS];
  __shared__ long long si[NTS];
  const int tid = threadIdx.x;
  double best = -1.0;
  long long bi = LLONG_MAX;
  for (int p = tid; p < nparts; p += NTS)
    if (beats(pv[p], pi[p], best, bi)) {
      best = pv[p];
      bi = pi[p];
    }
  block_argmax(best, bi, sv, si);
  const long long p = bi;
  if (tid == 0) {
    piv[k] = (int)p;
    w[p] = -1.0;  // never chosen again
  }
  for (int i = tid; i < n; i += NTS) a[i] = psi[(long long)i * nr + p];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = tid; j < k; j += NTS) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += qm[(long long)j * n + i] * a[i];
      c[j] = s;
    }
    __syncthreads();
    for (int i = tid; i < n; i += NTS) {
      double s = a[i];
      for (int j = 0; j < k; ++j) s -= c[j] * qm[(long long)j * n + i];
      a[i] = s;
    }
    __syncthreads();
  }
  double s2 = 0.0;
  for (int i = tid; i < n; i += NTS) s2 += a[i] * a[i];
  sv[tid] = s2;
  __syncthreads();
  for (int s = NTS / 2; s > 0; s >>= 1) {
    if (tid < s) sv[tid] += sv[tid + s];
    __syncthreads();
  }
  const double nrm = sv[0];
  const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : NAN;
  for (int i = tid; i < n; i += NTS) qm[(long long)k * n + i] = a[i] * inv;
}

// b[k][i] = psi_i(c_k)
__global__ void __launch_bounds__(NTS) k_scdm_gather(const double* __restrict__ psi, int n,
                                                      long long nr, const int* __restrict__ piv,
                                                      double* __restrict__ b) {
  const long long e = (long long)blockIdx.x * NTS + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int k = (int)(e / n), i = (int)(e - (long long)k * n);
  b[e] = psi[(long long)i * nr + piv[k]];
}

size_t scdm_scratch_bytes(long long nr) {
  return (size_t)nr * 8 + (size_t)kScdmParts * 16 + 256;
}

void launch_scdm_pivots(const double* psi, int n, long long nr, char* scratch, double* qm,
                        int* piv, hipStream_t st) {
  double* w = reinterpret_cast<double*>(scratch);
  char* tail = scratch + (((size_t)nr * 8 + 255) & ~(size_t)255);
  double* pv = reinterpret_cast<double*>(tail);
  long long* pi = reinterpret_cast<long long*>(tail + (size_t)kScdmParts * 8);
  hipLaunchKernelGGL(k_scdm_norms, dim3(kScdmParts), dim3(NTS), 0, st, psi, n, nr, w, pv, pi);
  const size_t pick_lds = (size_t)2 * n * 8;
  const size_t upd_lds = (size_t)n * 8;
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_scdm_pick, dim3(1), dim3(NTS), pick_lds, st, pv, pi, kScdmParts, psi, n,
                       nr, k, qm, piv, w);
    if (k + 1 < n)
      hipLaunchKernelGGL(k_scdm_update, dim3(kScdmParts), dim3(NTS), upd_lds, st, psi, n, nr,
                         qm + (size_t)k * n, w, pv, pi);
  }
}

void launch_scdm_gather(const double* psi, int n, long long nr, const int* piv, double* b,
                        hipStream_t st) {
  const long long tot = (long long)n * n;
  hipLaunchKernelGGL(k_scdm_gather, dim3((unsigned)((tot + NTS - 1) / NTS)), dim3(NTS), 0, st,
                     psi, n, nr, piv, b);
}

}  // namespace hfx
