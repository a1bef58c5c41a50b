// Elementwise helpers of the exchange pipeline: float64 -> float32 staging
// of the orbitals, zero fill (a kernel rather than a memset, so the calls stay
// graph-capture friendly), and the fixed-order float64 energy reduction.
#include <hip/hip_runtime.h>

#include "hfx_internal.hpp"

namespace hfx {

__global__ void __launch_bounds__(256) k_cast_f64_f32(const double* __restrict__ in,
                                                      float* __restrict__ out, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x * 2;
  for (size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; i < n; i += stride) {
    if (i + 1 < n) {
      const double2 v = *reinterpret_cast<const double2*>(in + i);
      *reinterpret_cast<float2*>(out + i) = make_float2((float)v.x, (float)v.y);
    } else {
      out[i] = (float)in[i];
    }
  }
}

__global__ void __launch_bounds__(256) k_zero(uint4* __restrict__ p, size_t n16,
                                              unsigned char* __restrict__ tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0)
    for (size_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

// out[0] = scale * sum(partials) + dc_scale * sum(mean^2), summed in a fixed
// order by one workgroup.  The second term is the G = 0 part of the pair
// energies when the pair-density means were taken out of the transforms.
// One workgroup; each thread keeps U independent partial sums (loads in
// flight together) combined in a fixed order, then a fixed tree: the result
// is bitwise reproducible.
__global__ void __launch_bounds__(1024) k_energy_reduce(const double* __restrict__ partials,
                                                        long long n, double scale,
                                                        const double* __restrict__ mean,
                                                        long long nmean, double dc_scale,
                                                        double* __restrict__ out) {
  constexpr int NT = 1024, U = 8;
  __shared__ double red[NT];
  const int tid = threadIdx.x;
  auto sum = [&](const double* v, long long len, bool square) {
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0.0;
    for (long long i0 = 0; i0 < len; i0 += (long long)NT * U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long i = i0 + tid + (long long)NT * u;
        const double x = i < len ? v[i] : 0.0;
        acc[u] += square ? x * x : x;
      }
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) s += acc[u];
    return s;
  };
  const double s = sum(partials, n, false);
  const double d = mean ? sum(mean, nmean, true) : 0.0;
  red[tid] = scale * s + dc_scale * d;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[0] = red[0];
}

template <typename S>
__global__ void __launch_bounds__(256) k_scale_to_f64(const S* __restrict__ src,
                                                      double* __restrict__ dst, size_t n,
                                                      double scale,
                                                      const double* __restrict__ gscale) {
  const double f = gscale ? scale * gscale[0] : scale;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = f * (double)src[i];
}

__global__ void __launch_bounds__(256) k_mask(double* __restrict__ m,
                                             const unsigned char* __restrict__ keep, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !keep[i]) m[i] = 0.0;
}

static int grid_for(size_t work) {
  const size_t b = (work + 255) / 256;
  return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

void launch_mask(double* m, const unsigned char* keep, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, m, keep, n);
}

void launch_cast_f64_f32(const double* in, float* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f64_f32, dim3(grid_for((n + 1) / 2)), dim3(256), 0, s, in, out, n);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  // buffers come from the caller; only the 16-byte body is vectorised
  const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
  if (addr % 16 != 0) {
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, static_cast<uint4*>(nullptr), (size_t)0,
                       static_cast<unsigned char*>(p), bytes);
    return;
  }
  const size_t n16 = bytes / 16;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(n16)), dim3(256), 0, s, static_cast<uint4*>(p), n16,
                     static_cast<unsigned char*>(p) + n16 * 16, bytes - n16 * 16);
}

void launch_scale_to_f64(const void* src, int src_is_f64, double* dst, size_t n, double scale,
                         const double* gscale, hipStream_t s) {
  if (src_is_f64)
    hipLaunchKernelGGL(k_scale_to_f64<double>, dim3(grid_for(n)), dim3(256), 0, s,
                       static_cast<const double*>(src), dst, n, scale, gscale);
  else
    hipLaunchKernelGGL(k_scale_to_f64<float>, dim3(grid_for(n)), dim3(256), 0, s,
                       static_cast<const float*>(src), dst, n, scale, gscale);
}

void launch_energy_reduce(const double* partials, long long n, double scale, const double* mean,
                          int n_orb, double dc_scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(1024), 0, s, partials, n, scale, mean,
                     (long long)n_orb * n_orb, dc_scale, out);
}

}  // namespace hfx
