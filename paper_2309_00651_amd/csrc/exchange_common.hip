// Elementwise helpers of the exchange pipeline: float64 -> float32 staging
// of the orbitals, zero fill (a kernel rather than a memset, so the calls stay
// graph-capture friendly), the fixed-order float64 energy reduction, and the
// optional input check (non-finite values, z band of the orbitals).
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

// Input check of 32 lines of psi along one axis: the number of non-finite
// values, sum psi^2, and, when m_max >= 0, the power of the spectrum beyond
// |m| <= m_max, sum over those k of |sum_z psi(z) e^(-2 pi i k z / len)|^2
// (len times its share of sum psi^2, by Parseval).  Direct DFT of the pruned
// frequencies from a line block in LDS: a check, not a hot path.  One
// 64-thread workgroup: 32 lines, two halves splitting points and
// frequencies; a fixed-order wavefront sum.
constexpr int kCheckXC = 32, kCheckNZ = 128;
// Lines of psi along one axis, 32 per workgroup (two halves of 32 threads
// share the points of a line): line l of orbital o starts at
// o * ostride + u * so + l * sl (u < no: the third axis) and has len points
// at stride sa.  Each thread sums its line's squares, counts non-finite
// values, and forms the direct DFT of the line at the frequencies |m| > m_max
// (m_max < 0: none), summing their power.
__global__ void __launch_bounds__(64) k_check_orbitals(const double* __restrict__ psi,
                                                      long long ostride, int len, long long sa,
                                                      int nl, long long sl, int no, long long so,
                                                      int m_max, double* __restrict__ part) {
  __shared__ double col[kCheckNZ][kCheckXC + 1];
  __shared__ double twc[kCheckNZ], tws[kCheckNZ];
  const int lcs = (nl + kCheckXC - 1) / kCheckXC;
  const long long b = blockIdx.x;
  const int lc = (int)(b % lcs);
  const int u = (int)((b / lcs) % no);
  const long long o = b / ((long long)lcs * no);
  const int t = threadIdx.x, c = t & (kCheckXC - 1), h = t >> 5;
  const int l = lc * kCheckXC + c;
  const bool valid = l < nl;
  const long long base = o * ostride + u * so + (valid ? l : 0) * sl;
  double tot = 0.0, bad = 0.0, oob = 0.0;
  for (int z = h; z < len; z += 2) {
    const double v = valid ? psi[base + z * sa] : 0.0;
    col[z][c] = v;
    tot += v * v;
    bad += isfinite(v) ? 0.0 : 1.0;
  }
  for (int k = t; k < len; k += 64) {
    double sn, cs;
    sincospi(-2.0 * k / len, &sn, &cs);
    twc[k] = cs;
    tws[k] = sn;
  }
  __syncthreads();
  if (m_max >= 0 && valid) {
    for (int k = m_max + 1 + h; k <= len - 1 - m_max; k += 2) {
      double re = 0.0, im = 0.0;
      int idx = 0;  // k z mod len
      for (int z = 0; z < len; ++z) {
        re += col[z][c] * twc[idx];
        im += col[z][c] * tws[idx];
        idx += k;
        if (idx >= len) idx -= len;
      }
      oob += re * re + im * im;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    tot += __shfl_xor(tot, off);
    bad += __shfl_xor(bad, off);
    oob += __shfl_xor(oob, off);
  }
  if (t == 0) {
    part[3 * b] = bad;
    part[3 * b + 1] = tot;
    part[3 * b + 2] = oob;
  }
}

// Geometry of the lines along axis a (0 x, 1 y, 2 z) of a [z][y][x] orbital:
// the lanes of a workgroup take neighbouring x (axes y and z) or y (axis x).
struct CheckAxis {
  int len, nl, no;
  long long sa, sl, so;
};
static CheckAxis check_axis(int a, int nx, int ny, int nz) {
  const long long nxy = (long long)nx * ny;
  if (a == 2) return {nz, nx, ny, nxy, 1, nx};
  if (a == 1) return {ny, nx, nz, nx, 1, nxy};
  return {nx, ny, nz, 1, nx, nxy};
}

long long check_partials(int n_orb, int nx, int ny, int nz, int axis) {
  const CheckAxis g = check_axis(axis, nx, ny, nz);
  return (long long)n_orb * g.no * ((g.nl + kCheckXC - 1) / kCheckXC);
}

bool launch_check_orbitals(const double* psi, int n_orb, int nx, int ny, int nz, int axis,
                           int m_max, double* part, hipStream_t s) {
  const CheckAxis g = check_axis(axis, nx, ny, nz);
  if (g.len > kCheckNZ) return false;
  hipLaunchKernelGGL(k_check_orbitals, dim3((unsigned)check_partials(n_orb, nx, ny, nz, axis)),
                     dim3(64), 0, s, psi, (long long)nx * ny * nz, g.len, g.sa, g.nl, g.sl, g.no,
                     g.so, m_max, part);
  return true;
}

// Grouped forms for the systems of a size class: segment s (count <=
// kMaxGroup) owns the workgroups [start[s], start[s + 1]) and walks its own
// range with a grid stride of its own workgroups.
struct SegGroup {
  const void* src[kMaxGroup];
  void* dst[kMaxGroup];
  size_t n[kMaxGroup];
  int start[kMaxGroup + 1];
  int count;
};
__device__ __forceinline__ int seg_locate(const SegGroup& g, int b, int& s) {
  int k = 0;
#pragma unroll
  for (int i = 1; i < kMaxGroup; ++i)
    if (i < g.count && b >= g.start[i]) k = i;
  s = k;
  return b - g.start[k];
}

__global__ void __launch_bounds__(256) k_cast_group(SegGroup g) {
  int s = 0;
  const int b = seg_locate(g, (int)blockIdx.x, s);
  const double* __restrict__ in = static_cast<const double*>(g.src[s]);
  float* __restrict__ out = static_cast<float*>(g.dst[s]);
  const size_t n = g.n[s];
  const size_t stride = (size_t)(g.start[s + 1] - g.start[s]) * blockDim.x * 2;
  for (size_t i = ((size_t)b * blockDim.x + threadIdx.x) * 2; i < n; i += stride) {
    if (i + 1 < n) {
      const double2 v = *reinterpret_cast<const double2*>(in + i);
      *reinterpret_cast<float2*>(out + i) = make_float2((float)v.x, (float)v.y);
    } else {
      out[i] = (float)in[i];
    }
  }
}

// byte ranges; n counts bytes
__global__ void __launch_bounds__(256) k_zero_group(SegGroup g) {
  int s = 0;
  const int b = seg_locate(g, (int)blockIdx.x, s);
  unsigned char* p = static_cast<unsigned char*>(g.dst[s]);
  const size_t bytes = g.n[s];
  const size_t stride = (size_t)(g.start[s + 1] - g.start[s]) * blockDim.x;
  const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
  const size_t head = addr % 16 ? (16 - addr % 16 < bytes ? 16 - addr % 16 : bytes) : 0;
  const size_t n16 = (bytes - head) / 16;
  uint4* body = reinterpret_cast<uint4*>(p + head);
  for (size_t i = (size_t)b * blockDim.x + threadIdx.x; i < n16; i += stride)
    body[i] = make_uint4(0u, 0u, 0u, 0u);
  if (b == 0) {
    for (size_t i = threadIdx.x; i < head; i += blockDim.x) p[i] = 0;
    for (size_t i = head + n16 * 16 + threadIdx.x; i < bytes; i += blockDim.x) p[i] = 0;
  }
}

static int grid_for(size_t work);

void launch_cast_group(const double* const* in, float* const* out, const size_t* n, int count,
                       hipStream_t s) {
  SegGroup g{};
  g.count = count;
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    g.src[i] = in[i];
    g.dst[i] = out[i];
    g.n[i] = n[i];
    g.start[i] = blocks;
    blocks += grid_for((n[i] + 1) / 2);
  }
  g.start[count] = blocks;
  hipLaunchKernelGGL(k_cast_group, dim3(blocks), dim3(256), 0, s, g);
}

void launch_zero_group(void* const* p, const size_t* bytes, int count, hipStream_t s) {
  SegGroup g{};
  g.count = count;
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    g.dst[i] = p[i];
    g.n[i] = bytes[i];
    g.start[i] = blocks;
    blocks += grid_for(bytes[i] / 16 > 0 ? bytes[i] / 16 : 1);
  }
  g.start[count] = blocks;
  hipLaunchKernelGGL(k_zero_group, dim3(blocks), dim3(256), 0, s, g);
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
