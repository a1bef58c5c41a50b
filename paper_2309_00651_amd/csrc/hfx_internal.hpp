// Internal interface between the host-side plan (hfx_api.cpp) and the
// templated HIP kernels (exchange_*.hip, gemm.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hfx {

// One orbital tile: pairs (a, b) with a in [i0, i0+nI) and b in [j0, j0+nJ).
// Off-diagonal tiles (diag == 0, disjoint blocks) take every (a, b); diagonal
// tiles (J inside I's block) take a <= b.  Packed pair-grid slot of
// (a - i0, b - j0) is slot0 + (a - i0) * (tile / 2) + (b - j0) / 2: the two
// pairs (a, 2p) and (a, 2p+1) share one complex grid (real and imaginary part).
// Most rows a tile pair may have: the pass kernels stage kMaxRows x tile pair
// means in LDS.
constexpr int kMaxRows = 32;

// One tile pair: rows i0..i0+nI-1 (I, up to kMaxRows) and columns
// j0..j0+nJ-1 (J, one tile of `tile` orbitals) in the plan's orbital order
// (see PassArgs::perm).  diag when both lie in one diagonal block of the
// schedule: J starts joff = j0 - i0 rows into I and only pairs i <= j are
// evaluated (row a, column b with a <= b + joff).  slot0 = first pair-grid
// slot.  keep0..keep3: bit 8 (a % 8) + b of word a / 8 set when the pair
// (row a, column b) is evaluated (all set unless the pairs are screened;
// screening needs 8-orbital column tiles).  Named words, not an array: a
// kernel's copy of the descriptor then stays in registers.
struct TileDesc {
  int i0, nI, j0, nJ, diag, joff, slot0;
  unsigned long long keep0, keep1, keep2, keep3;
};
static_assert(kMaxRows == 32, "four 64-bit mask words");

// Mask word w (rows 8 w .. 8 w + 7) of a tile pair, combined from values
// (a select between the fields' addresses would put the descriptor in memory).
__host__ __device__ inline unsigned long long keep_word(const TileDesc& td, int w) {
  const unsigned long long m0 = 0ull - (unsigned long long)(w == 0);
  const unsigned long long m1 = 0ull - (unsigned long long)(w == 1);
  const unsigned long long m2 = 0ull - (unsigned long long)(w == 2);
  const unsigned long long m3 = 0ull - (unsigned long long)(w == 3);
  return (td.keep0 & m0) | (td.keep1 & m1) | (td.keep2 & m2) | (td.keep3 & m3);
}

// Arguments of one exchange pass over one batch of tiles of one system.
struct PassArgs {
  const void* psi;        // [n_orb][N^3] orbitals in the working precision
  void* kpsi;             // [n_orb][N^3] K psi accumulators (working precision)
  void* grids;            // [slots][N^3] complex pair grids
  const TileDesc* tiles;  // tiles of this batch
  const int* active;      // grid slots that carry at least one pair
  const void* vtab;       // v(G) / N_r, [kz][ky][kx]
  const void* tw_zf;      // twiddle tables (see twiddle.hpp) per axis/direction
  const void* tw_zi;
  const void* tw_xf;
  const void* tw_xi;
  const void* tw_yf;
  const void* tw_yi;
  const void* tw_zh;      // forward z at half length (band-limited to a quarter of NZ), or null
  double* partials;       // per-workgroup energy partial sums
  long long part_base;    // first partial of this launch
  const double* mean;     // float32 plans: pair-density means mu_ab = (1/N_r) sum psi_a psi_b
                          // (n_orb x n_orb), subtracted before the forward FFT; else null
  double v0;              // v(G = 0), re-added to the potentials as v0 * mu_ab
  const int* perm;        // orbital at each position of the tile order (null: identity)
  int n_orb;
  int n_tiles;
  int n_active;
  // Band-limited orbitals: pair densities vanish on the kz planes with
  // |kz| > kz_max, which are then neither stored, transformed nor loaded
  // (read as zeros).  kz_max >= NZ / 2: every plane is kept.
  int kz_max;
  const void* zero;  // kZeroBytes of zeros (device): the pruned planes' loads read these
  // Band-limited orbitals: pair densities also vanish for |kx| > kx_max, so
  // the plane pass may skip the y transforms of those columns (kx_max >=
  // N / 2: every column is kept).
  int kx_max;
  int ky_max;  // the same along y
};

// Zero block of band-limited plans (the pruned planes' loads read its first
// element).
constexpr int kZeroBytes = 1024 * 16;

// Whether z frequency index k (0 <= k < nz) lies on a kept plane.
__host__ __device__ inline bool kz_kept(int k, int nz, int kz_max) {
  return (k <= nz - k ? k : nz - k) <= kz_max;
}
// Number of kept kz planes, and the frequency index of compact plane c
// (0 <= c < kz_planes): 0 .. kz_max, then nz - kz_max .. nz - 1.  Written
// without 2 kz_max, which overflows for the "keep all" value.
__host__ __device__ inline int kz_planes(int nz, int kz_max) {
  return kz_max >= nz / 2 ? nz : 2 * kz_max + 1;
}
__host__ __device__ inline int kz_of_plane(int c, int nz, int kz_max) {
  return (kz_max >= nz / 2 || c <= kz_max) ? c : nz - (2 * kz_max + 1 - c);
}

// One launch of a pass over the current batches of up to kMaxGroup systems
// that share a kernel configuration (a size class): system s owns the
// logical workgroups [start[s], start[s + 1]) and reads its own PassArgs.
// Single-system launches are groups of one.  Passed by value as the kernel
// argument (about 1.3 KB), so a launch needs no device-side table upload
// and can be captured in a graph as is.
constexpr int kMaxGroup = 8;
struct PassGroup {
  PassArgs a[kMaxGroup];
  int start[kMaxGroup + 1];
  int count;
  // system of logical workgroup L (in s) and L's index inside that system
  __device__ __forceinline__ int locate(int L, int& s) const {
    int k = 0;
#pragma unroll
    for (int i = 1; i < kMaxGroup; ++i)
      if (i < count && L >= start[i]) k = i;
    s = k;
    return L - start[k];
  }
};

typedef void (*launch_fn)(const PassGroup&, int nblocks, hipStream_t);

// One compiled configuration of the exchange pipeline for a grid size and
// precision: radix schedules, launch shapes and the launchers.
struct Variant {
  const char* name;
  int n;           // grid points along x and y
  int nz;          // grid points along z (n for cubic grids)
  int prec;        // 0 float32, 1 float64
  int brick;       // pencil width W (x values per workgroup)
  int tile;        // orbital tile T (columns of a tile pair)
  int max_rows;    // most rows per tile pair (T when psi of I is staged in LDS)
  int nt_fwd;      // threads per pair_fwd workgroup
  int nt_acc;      // threads per inv_acc workgroup
  int nt_plane;    // threads per plane workgroup (plane_mode 1: per row workgroup)
  int nt_cols;     // plane_mode 1: threads per column workgroup
  int plane_mode;  // 0: fused xy plane in LDS; 1: x rows + y columns passes
  int rows_per_wg; // plane_mode 1: rows per row-FFT workgroup
  bool persistent; // plane kernel loops over planes (grid of resident workgroups only)
  int zf[4], nzf, zi[4], nzi;  // z radix schedules (forward, inverse)
  int zh[4], nzh;              // forward z at half length (nzh = 0: not compiled)
  int qb;                      // band columns of the plane kernel (|kx| <= qb), 0: none
  bool hy;                     // half-height plane input compiled (band-limited y)
  bool xd;                     // half-width plane input compiled too (band-limited x)
  int xf[4], nxf, xi[4], nxi;  // x
  int yf[4], nyf, yi[4], nyi;  // y
  size_t plane_lds;            // dynamic LDS bytes of the plane/row kernels
  launch_fn pair_fwd;          // pair product + forward z FFT
  launch_fn plane;             // plane_mode 0: x/y forward, * v, y/x inverse
  launch_fn rows_fwd;          // plane_mode 1: forward x FFT on rows
  launch_fn cols_conv;         // plane_mode 1: y forward, * v, y inverse
  launch_fn rows_inv;          // plane_mode 1: inverse x FFT on rows
  launch_fn inv_acc;           // inverse z FFT + energy + K psi accumulation
  launch_fn inv_energy;        // inverse z FFT + energy only
  hipError_t (*prepare)();     // raise dynamic-LDS limits of the kernels
};

const Variant* variants_f32(int* count);
const Variant* variants_f64(int* count);

// Elementwise helpers (exchange_common.hip)
void launch_cast_f64_f32(const double* in, float* out, size_t n, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);
// m[i] = keep[i] ? m[i] : 0 (n values)
void launch_mask(double* m, const unsigned char* keep, size_t n, hipStream_t s);
// grad[i] = scale * gscale[0 or nothing] * src[i] (src float32 or float64, in place allowed
// for float64)
void launch_scale_to_f64(const void* src, int src_is_f64, double* dst, size_t n, double scale,
                         const double* gscale, hipStream_t s);
// out[0] = scale * sum(partials) + dc_scale * sum_ab mean[a][b]^2 (mean: n x n, nullable)
void launch_energy_reduce(const double* partials, long long n, double scale, const double* mean,
                          int n_orb, double dc_scale, double* out, hipStream_t s);

// The same for the count <= kMaxGroup systems of a size class in one launch
// each: out[i] <- in[i] (n[i] values), p[i] zeroed (bytes[i] bytes).
void launch_cast_group(const double* const* in, float* const* out, const size_t* n, int count,
                       hipStream_t s);
void launch_zero_group(void* const* p, const size_t* bytes, int count, hipStream_t s);

// Input check (exchange_common.hip) along axis 0 (x), 1 (y) or 2 (z): per
// (orbital, index along a third axis, chunk of 32 lines) three doubles:
// non-finite count, sum psi^2, power of the spectrum along the axis beyond
// |m| <= m_max (m_max < 0: not computed).  check_partials() triples of
// output; false (nothing launched) for an axis longer than 128.
long long check_partials(int n_orb, int nx, int ny, int nz, int axis);
bool launch_check_orbitals(const double* psi, int n_orb, int nx, int ny, int nz, int axis,
                           int m_max, double* part, hipStream_t s);

// Dense products (gemm.hip); `partial` holds gemm_partial_bytes(n_orb, nr).
// C[k][l] = alpha * sum_r A[k][r] B[l][r], A float64 split into hi + lo
// float32 parts, B float32, float32 MFMA with float64 accumulation across
// k-blocks; partials then reduced in a fixed order.
void launch_xtx_split(const double* a, const float* b, int n_orb, long long nr, double alpha,
                      double* partial, double* c, hipStream_t s);
// C = alpha * A B^T with A, B float64 [n][nr] (float64 MFMA; a == b: symmetric)
void launch_xtx_f64(const double* a, const double* b, int n_orb, long long nr, double alpha,
                    double* partial, double* c, hipStream_t s);
// C = alpha |A| |A|^T (float64 MFMA, symmetric)
void launch_xtx_abs(const double* a, int n_orb, long long nr, double alpha, double* partial,
                    double* c, hipStream_t s);
size_t gemm_partial_bytes(int n_orb, long long nr);
// C_i = alpha_i A_i A_i^T (float64 MFMA, symmetric) for count <= kMaxGroup
// products in one launch of the product and one of the reduction; each
// result equals launch_xtx_f64's for the same arguments bit for bit.
void launch_gram_self_group(const double* const* a, const int* n, const long long* nr,
                            const double* alpha, double* const* part, double* const* c,
                            int count, hipStream_t s);

// Orthonormalisation helpers (ortho.hip)
hipError_t launch_inverse_sqrt(double* s, int n, double* work, int max_iter, hipStream_t st);
void launch_apply_left(const double* m, const double* src, double* dst, int n, long long nr,
                       double* tmp, hipStream_t st);
// dst <- m widen(src), float32 src (n <= 512; false otherwise, nothing launched)
bool launch_apply_left_f32(const double* m, const float* src, double* dst, int n, long long nr,
                           hipStream_t st);
hipError_t prepare_apply_left();

// SCDM pivot selection (scdm.hip)
constexpr int kScdmParts = 2048;  // workgroups of the grid-wide passes
size_t scdm_scratch_bytes(long long nr);
// piv[k] (k < n) = grid points chosen by column-pivoted QR of psi^T (n x nr);
// scratch: scdm_scratch_bytes(nr); qm: n x n doubles (rows q_k)
void launch_scdm_pivots(const double* psi, int n, long long nr, char* scratch, double* qm,
                        int* piv, hipStream_t st);
// b[k][i] = psi[i][piv[k]]
void launch_scdm_gather(const double* psi, int n, long long nr, const int* piv, double* b,
                        hipStream_t st);

// Cholesky helpers (ace.hip): l = lower Cholesky factor of sign * m; x = l^(-1)
void launch_chol(const double* m, int n, double sign, double* l, hipStream_t s);
void launch_trinv(const double* l, int n, double* x, hipStream_t s);

}  // namespace hfx
