// Exchange pipeline kernels (templated on precision, grid size and schedules).
//
// One "pair grid" packs two real pair densities as one complex grid,
// c = psi_a psi_b + i psi_a psi_b'.  Because v(G) is real and even, the
// real and imaginary parts of IFFT(v FFT(c)) are the two pair potentials
// v_ab and v_ab' of Eq. (vij) (Methods, MTACE subsection).
//
// Three passes per batch of tiles, all over workspace grids [slot][z][y][x]:
//   pair_fwd : a brick of W x-columns at fixed y, all z: forms the products
//              from psi (read once per tile), forward FFT along z, stores.
//   plane    : one kz plane of one grid: forward FFT along x and y in LDS,
//              multiply by v(G)/N_r, inverse along y and x, stores.
//              (float64 grids whose plane exceeds LDS use rows_fwd,
//              cols_conv and rows_inv instead.)
//   inv_acc  : the brick again: inverse FFT along z, then per point the pair
//              energies rho_ab v_ab (float64 sums) and
//              K psi_a -= v_ab psi_b, K psi_b -= v_ab psi_a   (Eq. vx).
// Workgroups of one launch touch disjoint K psi rows (tiles of a batch share
// no orbital, bricks of a tile share no point), so accumulation is plain
// read-modify-write with a fixed order: results are bitwise reproducible.
#pragma once

#include "fft.hpp"
#include "hfx_internal.hpp"

namespace hfx {

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD walks a contiguous range of logical indices (shared L2 for neighbours).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Deterministic workgroup sum of one double per thread (fixed tree order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  constexpr int P2 = NT <= 64 ? 64 : NT <= 128 ? 128 : NT <= 256 ? 256 : NT <= 512 ? 512 : 1024;
  red[tid] = v;
  for (int t = tid + NT; t < P2; t += NT) red[t] = 0.0;
  __syncthreads();
#pragma unroll
  for (int s = P2 / 2; s > 0; s >>= 1) {
    for (int t = tid; t < s; t += NT) red[t] += red[t + s];
    __syncthreads();
  }
  return red[0];
}

template <int NT>
constexpr int pow2_at_least() {
  return NT <= 64 ? 64 : NT <= 128 ? 128 : NT <= 256 ? 256 : NT <= 512 ? 512 : 1024;
}

// ---------------------------------------------------------------------------
// Pass 1: pair product + forward z FFT on bricks.
// Two pair grids are transformed together: LDS holds [z][2W] with the brick
// of grid g in columns [gW, gW + W).  Thread tid forms the products at brick
// points p = tid + k NT (k < PT, contiguous x for coalesced psi reads) for both
// grids; the transform starts from LDS and its last stage stores straight to
// HBM.  psi of the tile's J block stays in registers for the whole tile.
template <typename T, int N, int W, int NT, int TT, class SZF>
__global__ void __launch_bounds__(NT) k_pair_fwd(PassArgs a) {
  static_assert(TT % 4 == 0, "tile must hold whole grid pairs");
  constexpr int W2 = 2 * W;
  using G = Geom<T, N, W2, NT, true, W2, 1>;
  using L = LastStage<G, SZF>;
  using E = FFT<G, false, SZF>;
  constexpr int RL = SchedInfo<SZF>::last;
  constexpr int NXB = (N + W - 1) / W;
  constexpr int BR = N * NXB;
  constexpr int P = N * W;
  constexpr int PT = (P + NT - 1) / NT;
  constexpr long long NR = (long long)N * N * N;
  constexpr int ZSL = (N / RL) * N * N;  // offset between legs of a last-stage butterfly
  __shared__ cpx<T> lds[N * W2];
  const int tid = threadIdx.x;
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const int t = lg / BR, br = lg - t * BR;
  const int y = br / NXB, x0 = (br - y * NXB) * W;
  const TileDesc td = a.tiles[t];
  const T* __restrict__ psi = static_cast<const T*>(a.psi);
  const TwEntry<T>* __restrict__ tw = static_cast<const TwEntry<T>*>(a.tw_zf);
  cpx<T>* __restrict__ grids = static_cast<cpx<T>*>(a.grids);

  int offA[PT], ldsA[PT];
  bool vA[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int p = tid + k * NT;
    const int z = p / W, m = p - (p / W) * W;
    vA[k] = p < P && (x0 + m) < N;
    offA[k] = vA[k] ? (z * N + y) * N + x0 + m : 0;
    ldsA[k] = z * W2 + m;
  }
  int offL[L::PER], gL[L::PER];
  bool vL[L::PER];
#pragma unroll
  for (int i = 0; i < L::PER; ++i) {
    int m = 0, j = 0;
    L::mj(tid, i, m, j);
    gL[i] = m / W;
    const int mx = m - gL[i] * W;
    vL[i] = L::valid(tid, i) && (x0 + mx) < N;
    offL[i] = vL[i] ? (j * N + y) * N + x0 + mx : 0;
  }

  T pj[TT][PT];
#pragma unroll
  for (int b = 0; b < TT; ++b) {
    const bool bv = b < td.nJ;
    const T* p = psi + (long long)(td.j0 + (bv ? b : 0)) * NR;
#pragma unroll
    for (int k = 0; k < PT; ++k) pj[b][k] = (bv && vA[k]) ? p[offA[k]] : T(0);
  }

  for (int ia = 0; ia < td.nI; ++ia) {
    const T* pa_ptr = psi + (long long)(td.i0 + ia) * NR;
    T pa[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) pa[k] = vA[k] ? pa_ptr[offA[k]] : T(0);
    static_for<0, TT / 4>([&](auto bq) {
      constexpr int b0 = 4 * decltype(bq)::value;  // pairs (a, b0 .. b0 + 3), grids 2bq, 2bq+1
      // grid g carries pairs (a, b0 + 2g) and (a, b0 + 2g + 1)
      const bool use0 = b0 < td.nJ && !(td.diag && b0 + 1 < ia);
      const bool use1 = b0 + 2 < td.nJ && !(td.diag && b0 + 3 < ia);
      if (!use0 && !use1) return;
      // pair-density means (float32 plans): transforms see zero-mean densities
      T mu[4] = {T(0), T(0), T(0), T(0)};
      if (a.mean) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (b0 + q < td.nJ) mu[q] = (T)a.mean[(long long)(td.i0 + ia) * a.n_orb + td.j0 + b0 + q];
      }
#pragma unroll
      for (int k = 0; k < PT; ++k)
        if (tid + k * NT < P) {
          const T in = vA[k] ? T(1) : T(0);  // columns beyond the grid stay zero
          lds[ldsA[k]] = {pa[k] * pj[b0][k] - in * mu[0], pa[k] * pj[b0 + 1][k] - in * mu[1]};
          lds[ldsA[k] + W] = {pa[k] * pj[b0 + 2][k] - in * mu[2],
                              pa[k] * pj[b0 + 3][k] - in * mu[3]};
        }
      __syncthreads();
      cpx<T> out[L::VALS];
      E::lds2reg(lds, tw, tid, out);
      const int slot0 = td.slot0 + ia * (TT / 2) + 2 * decltype(bq)::value;
#pragma unroll
      for (int i = 0; i < L::PER; ++i) {
        const bool use = gL[i] == 0 ? use0 : use1;
        if (vL[i] && use) {
          cpx<T>* g = grids + (long long)(slot0 + gL[i]) * NR;
#pragma unroll
          for (int r = 0; r < RL; ++r) g[offL[i] + r * ZSL] = out[i * RL + r];
        }
      }
    });
  }
}

// ---------------------------------------------------------------------------
// Pass 3: inverse z FFT + pair energies + K psi accumulation on bricks.
// Two pair grids are transformed together ([z][2W] in LDS, as in pass 1).
// The inverse transform leaves the potentials in LDS in natural order; the
// accumulation then uses its own point map: thread tid owns brick points
// p = tid + k NT (k < PT), contiguous x for coalesced K psi traffic.  psi of
// the tile's J block and the J-side accumulators stay in registers for the
// whole tile; the pair energy of a thread's points is summed in the working
// precision per pair and added to a float64 accumulator once per pair.
template <typename T, int N, int W, int NT, int TT, class SZI, bool ACC>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && N >= 64 && N <= 96) ? 4 : 1)))
k_inv_acc(PassArgs a) {
  static_assert(TT % 4 == 0, "tile must hold whole grid pairs");
  constexpr int W2 = 2 * W;
  using G = Geom<T, N, W2, NT, true, W2, 1>;
  using F = FirstStage<G, SZI>;
  using E = FFT<G, true, SZI>;
  constexpr int RF = SchedInfo<SZI>::first;
  constexpr int NXB = (N + W - 1) / W;
  constexpr int BR = N * NXB;
  constexpr int P = N * W;                 // brick points
  constexpr int PT = (P + NT - 1) / NT;    // accumulation points per thread
  constexpr long long NR = (long long)N * N * N;
  constexpr int ZSF = (N / RF) * N * N;    // offset between legs of a first-stage butterfly
  __shared__ cpx<T> lds[N * W2];
  __shared__ double red[pow2_at_least<NT>()];
  const int tid = threadIdx.x;
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const int t = lg / BR, br = lg - t * BR;
  const int y = br / NXB, x0 = (br - y * NXB) * W;
  const TileDesc td = a.tiles[t];
  const T* __restrict__ psi = static_cast<const T*>(a.psi);
  T* __restrict__ kpsi = static_cast<T*>(a.kpsi);
  const TwEntry<T>* __restrict__ tw = static_cast<const TwEntry<T>*>(a.tw_zi);
  const cpx<T>* __restrict__ grids = static_cast<const cpx<T>*>(a.grids);

  int offF[F::PER], gF[F::PER];
  bool vF[F::PER];
#pragma unroll
  for (int i = 0; i < F::PER; ++i) {
    int m = 0, j = 0;
    F::mj(tid, i, m, j);
    gF[i] = m / W;
    const int mx = m - gF[i] * W;
    vF[i] = F::valid(tid, i) && (x0 + mx) < N;
    offF[i] = vF[i] ? (j * N + y) * N + x0 + mx : 0;
  }
  int offA[PT], ldsA[PT];
  bool vA[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int p = tid + k * NT;
    const int z = p / W, m = p - (p / W) * W;
    vA[k] = p < P && (x0 + m) < N;
    offA[k] = vA[k] ? (z * N + y) * N + x0 + m : 0;
    ldsA[k] = z * W2 + m;
  }

  T pj[TT][PT];
  T accJ[ACC ? TT : 1][PT];
#pragma unroll
  for (int b = 0; b < TT; ++b) {
    const bool bv = b < td.nJ;
    const T* pb = psi + (long long)(td.j0 + (bv ? b : 0)) * NR;
#pragma unroll
    for (int k = 0; k < PT; ++k) pj[b][k] = (bv && vA[k]) ? pb[offA[k]] : T(0);
  }
#pragma unroll
  for (int b = 0; b < (ACC ? TT : 1); ++b)
#pragma unroll
    for (int k = 0; k < PT; ++k) accJ[b][k] = T(0);
  double eacc = 0.0;

  for (int ia = 0; ia < td.nI; ++ia) {
    const int oa = td.i0 + ia;
    const T* pa_ptr = psi + (long long)oa * NR;
    T pa[PT], acca[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      pa[k] = vA[k] ? pa_ptr[offA[k]] : T(0);
      acca[k] = T(0);
    }
    static_for<0, TT / 4>([&](auto bq) {
      constexpr int b0 = 4 * decltype(bq)::value;
      const bool use0 = b0 < td.nJ && !(td.diag && b0 + 1 < ia);
      const bool use1 = b0 + 2 < td.nJ && !(td.diag && b0 + 3 < ia);
      if (!use0 && !use1) return;
      const int slot0 = td.slot0 + ia * (TT / 2) + 2 * decltype(bq)::value;
      cpx<T> v[F::VALS];
#pragma unroll
      for (int i = 0; i < F::PER; ++i) {
        const bool use = gF[i] == 0 ? use0 : use1;
        const cpx<T>* g = grids + (long long)(slot0 + gF[i]) * NR;
#pragma unroll
        for (int r = 0; r < RF; ++r)
          v[i * RF + r] = (vF[i] && use) ? g[offF[i] + r * ZSF] : cpx<T>{T(0), T(0)};
      }
      {
        cpx<T> out[LastStage<G, SZI>::VALS];
        E::reg2reg(v, lds, tw, tid, out);
        E::store_last(out, lds, tid);
      }
      __syncthreads();
      // one grid's potentials at a time (bounded registers)
      cpx<T> pot[PT];
      static_for<0, 4>([&](auto q) {
        constexpr int gq = decltype(q)::value / 2, half = decltype(q)::value % 2;
        constexpr int b = b0 + decltype(q)::value;
        if constexpr (half == 0) {
#pragma unroll
          for (int k = 0; k < PT; ++k)
            pot[k] = tid + k * NT < P ? lds[ldsA[k] + gq * W] : cpx<T>{T(0), T(0)};
        }
        if (b >= td.nJ) return;
        if (!(gq == 0 ? use0 : use1)) return;
        // weight of e_ab in sum_{i,j} e_ij: 2 for a != b, 1 for a == b
        const int w = td.diag ? (b > ia ? 2 : (b == ia ? 1 : 0)) : 2;
        if (w == 0) return;
        // G = 0 part of v_ab when the mean was taken out of the transform;
        // its energy v0 * Omega * mu_ab^2 is added in float64 at the reduction
        const T dc = a.mean ? (T)(a.v0 * a.mean[(long long)oa * a.n_orb + td.j0 + b]) : T(0);
        T es = T(0);
#pragma unroll
        for (int k = 0; k < PT; ++k) {
          const T vz = half ? pot[k].im : pot[k].re;  // zero-mean part
          es += vz * pj[b][k] * pa[k];                        // rho_ab v_ab
          if constexpr (ACC) {
            const T vv = vz + dc;
            accJ[b][k] -= vv * pa[k];
            if (w == 2) acca[k] -= vv * pj[b][k];
          }
        }
        eacc += (double)w * (double)es;
      });
      __syncthreads();  // LDS is rewritten by the next transform
    });
    if constexpr (ACC) {
      T* ka = kpsi + (long long)oa * NR;
#pragma unroll
      for (int k = 0; k < PT; ++k)
        if (vA[k]) ka[offA[k]] += acca[k];
    }
  }
  if constexpr (ACC) {
#pragma unroll
    for (int b = 0; b < TT; ++b) {
      if (b >= td.nJ) break;
      T* kb = kpsi + (long long)(td.j0 + b) * NR;
#pragma unroll
      for (int k = 0; k < PT; ++k)
        if (vA[k]) kb[offA[k]] += accJ[b][k];
    }
  }
  const double s = block_sum<NT>(eacc, red);
  if (tid == 0) a.partials[a.part_base + lg] = s;
}

// ---------------------------------------------------------------------------
// Pass 2: fused plane convolution for one kz plane of one pair grid.
template <typename T, int N, int NT, class SXF, class SXI, class SYF, class SYI>
__global__ void __launch_bounds__(NT) k_plane_conv(PassArgs a) {
  constexpr int P = N + 1;
  using GX = Geom<T, N, N, NT, false, 1, P>;  // rows: sequence m = y, element n = x
  using GY = Geom<T, N, N, NT, true, P, 1>;   // columns: sequence m = x, element n = y
  using EXF = FFT<GX, false, SXF>;
  using EXI = FFT<GX, true, SXI>;
  using EYF = FFT<GY, false, SYF>;
  using EYI = FFT<GY, true, SYI>;
  using FX = FirstStage<GX, SXF>;
  using LXF = LastStage<GX, SXF>;
  using LY = LastStage<GY, SYF>;
  using FYI = FirstStage<GY, SYI>;
  using LYI = LastStage<GY, SYI>;
  using LXI = LastStage<GX, SXI>;
  static_assert(SchedInfo<SYI>::first == SchedInfo<SYF>::last, "fused y schedules");
  static_assert(FYI::VALS == LY::VALS, "fused y register maps");
  constexpr long long NR = (long long)N * N * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* plane = reinterpret_cast<cpx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const int kz = lg / a.n_active, ai = lg - kz * a.n_active;
  const int slot = a.active[ai];
  cpx<T>* __restrict__ base = static_cast<cpx<T>*>(a.grids) + (long long)slot * NR + (long long)kz * N * N;
  const T* __restrict__ vt = static_cast<const T*>(a.vtab) + (long long)kz * N * N;

  // x forward: stage-0 inputs straight from HBM (rows, x contiguous)
  cpx<T> v[FX::VALS];
#pragma unroll
  for (int i = 0; i < FX::PER; ++i) {
    if (!FX::valid(tid, i)) continue;
    int m, j;
    FX::mj(tid, i, m, j);
#pragma unroll
    for (int r = 0; r < SchedInfo<SXF>::first; ++r)
      v[i * SchedInfo<SXF>::first + r] = base[m * N + FX::in_pos(j, r)];
  }
  {
    cpx<T> o[LXF::VALS];
    EXF::reg2reg(v, plane, static_cast<const TwEntry<T>*>(a.tw_xf), tid, o);
    EXF::store_last(o, plane, tid);
  }
  __syncthreads();
  // y forward, multiply by v(G)/N_r, y inverse (hand-over in registers)
  cpx<T> oy[LY::VALS];
  EYF::lds2reg(plane, static_cast<const TwEntry<T>*>(a.tw_yf), tid, oy);
#pragma unroll
  for (int i = 0; i < LY::PER; ++i) {
    if (!LY::valid(tid, i)) continue;
    int m, j;
    LY::mj(tid, i, m, j);
#pragma unroll
    for (int r = 0; r < SchedInfo<SYF>::last; ++r) {
      const T f = vt[LY::in_pos(j, r) * N + m];
      oy[i * SchedInfo<SYF>::last + r] = cscale(oy[i * SchedInfo<SYF>::last + r], f);
    }
  }
  {
    cpx<T> o[LYI::VALS];
    EYI::reg2reg(oy, plane, static_cast<const TwEntry<T>*>(a.tw_yi), tid, o);
    EYI::store_last(o, plane, tid);
  }
  __syncthreads();
  // x inverse, results straight to HBM
  cpx<T> ox[LXI::VALS];
  EXI::lds2reg(plane, static_cast<const TwEntry<T>*>(a.tw_xi), tid, ox);
#pragma unroll
  for (int i = 0; i < LXI::PER; ++i) {
    if (!LXI::valid(tid, i)) continue;
    int m, j;
    LXI::mj(tid, i, m, j);
#pragma unroll
    for (int r = 0; r < SchedInfo<SXI>::last; ++r)
      base[m * N + LXI::in_pos(j, r)] = ox[i * SchedInfo<SXI>::last + r];
  }
}

// ---------------------------------------------------------------------------
// Split plane pass for grids whose plane does not fit in LDS:
// (a) FFT along x of RW consecutive rows, (b) y columns with the multiply.
template <typename T, int N, int RW, int NT, class SX, bool INV>
__global__ void __launch_bounds__(NT) k_rows(PassArgs a) {
  constexpr int P = N + 1;
  using G = Geom<T, N, RW, NT, false, 1, P>;
  using E = FFT<G, INV, SX>;
  using F = FirstStage<G, SX>;
  using L = LastStage<G, SX>;
  constexpr long long NR = (long long)N * N * N;
  constexpr int RB = (N * N + RW - 1) / RW;  // row blocks per grid
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const int ai = lg / RB, rb = lg - ai * RB;
  const int slot = a.active[ai];
  cpx<T>* __restrict__ base = static_cast<cpx<T>*>(a.grids) + (long long)slot * NR;
  const long long row0 = (long long)rb * RW;
  const TwEntry<T>* tw = static_cast<const TwEntry<T>*>(INV ? a.tw_xi : a.tw_xf);
  cpx<T> v[F::VALS];
#pragma unroll
  for (int i = 0; i < F::PER; ++i) {
    if (!F::valid(tid, i)) continue;
    int m, j;
    F::mj(tid, i, m, j);
    const bool rv = row0 + m < (long long)N * N;
#pragma unroll
    for (int r = 0; r < SchedInfo<SX>::first; ++r)
      v[i * SchedInfo<SX>::first + r] =
          rv ? base[(row0 + m) * N + F::in_pos(j, r)] : cpx<T>{T(0), T(0)};
  }
  cpx<T> o[L::VALS];
  E::reg2reg(v, lds, tw, tid, o);
#pragma unroll
  for (int i = 0; i < L::PER; ++i) {
    if (!L::valid(tid, i)) continue;
    int m, j;
    L::mj(tid, i, m, j);
    if (row0 + m >= (long long)N * N) continue;
#pragma unroll
    for (int r = 0; r < SchedInfo<SX>::last; ++r)
      base[(row0 + m) * N + L::in_pos(j, r)] = o[i * SchedInfo<SX>::last + r];
  }
}

template <typename T, int N, int W, int NT, class SYF, class SYI>
__global__ void __launch_bounds__(NT) k_cols_conv(PassArgs a) {
  using G = Geom<T, N, W, NT, true, W, 1>;
  using EF = FFT<G, false, SYF>;
  using EI = FFT<G, true, SYI>;
  using F = FirstStage<G, SYF>;
  using LF = LastStage<G, SYF>;
  using FI = FirstStage<G, SYI>;
  using LI = LastStage<G, SYI>;
  static_assert(SchedInfo<SYI>::first == SchedInfo<SYF>::last, "fused y schedules");
  static_assert(FI::VALS == LF::VALS, "fused y register maps");
  constexpr int NXB = (N + W - 1) / W;
  constexpr long long NR = (long long)N * N * N;
  __shared__ cpx<T> lds[N * W];
  const int tid = threadIdx.x;
  const int lg = xcd_remap(blockIdx.x, gridDim.x);
  const int per_grid = N * NXB;
  const int ai = lg / per_grid, rem = lg - ai * per_grid;
  const int z = rem / NXB, x0 = (rem - z * NXB) * W;
  const int slot = a.active[ai];
  cpx<T>* __restrict__ base = static_cast<cpx<T>*>(a.grids) + (long long)slot * NR + (long long)z * N * N;
  const T* __restrict__ vt = static_cast<const T*>(a.vtab) + (long long)z * N * N;
  cpx<T> v[F::VALS];
#pragma unroll
  for (int i = 0; i < F::PER; ++i) {
    int m = 0, j = 0;
    F::mj(tid, i, m, j);
    const bool ok = F::valid(tid, i) && x0 + m < N;
#pragma unroll
    for (int r = 0; r < SchedInfo<SYF>::first; ++r)
      v[i * SchedInfo<SYF>::first + r] =
          ok ? base[F::in_pos(j, r) * N + x0 + m] : cpx<T>{T(0), T(0)};
  }
  cpx<T> o[LF::VALS];
  EF::reg2reg(v, lds, static_cast<const TwEntry<T>*>(a.tw_yf), tid, o);
#pragma unroll
  for (int i = 0; i < LF::PER; ++i) {
    int m = 0, j = 0;
    LF::mj(tid, i, m, j);
    const bool ok = LF::valid(tid, i) && x0 + m < N;
#pragma unroll
    for (int r = 0; r < SchedInfo<SYF>::last; ++r) {
      const T f = ok ? vt[LF::in_pos(j, r) * N + x0 + m] : T(0);
      o[i * SchedInfo<SYF>::last + r] = cscale(o[i * SchedInfo<SYF>::last + r], f);
    }
  }
  cpx<T> b[LI::VALS];
  EI::reg2reg(o, lds, static_cast<const TwEntry<T>*>(a.tw_yi), tid, b);
#pragma unroll
  for (int i = 0; i < LI::PER; ++i) {
    int m = 0, j = 0;
    LI::mj(tid, i, m, j);
    if (!(LI::valid(tid, i) && x0 + m < N)) continue;
#pragma unroll
    for (int r = 0; r < SchedInfo<SYI>::last; ++r)
      base[LI::in_pos(j, r) * N + x0 + m] = b[i * SchedInfo<SYI>::last + r];
  }
}

// ---------------------------------------------------------------------------
// Registry glue: one compiled pipeline configuration.

// Brick points per thread of the pair_fwd / inv_acc passes: 4 in float32,
// 2 in float64 (keeps the tile's psi and accumulators in registers at >= 3-4
// wavefronts per SIMD), and 4 for float64 bricks too large for 768 threads
// (more threads per workgroup would cap the registers at 128 and spill).
template <typename T, int N, int W>
constexpr int pts_per_thread() {
  return sizeof(T) == 4 ? 4 : (N * W / 2 > 768 ? 4 : 2);
}
template <int... R>
constexpr void fill_radices(int* dst, int& n, Sched<R...>) {
  const int r[] = {R...};
  n = (int)sizeof...(R);
  for (int i = 0; i < n; ++i) dst[i] = r[i];
}

template <typename T, int N, int W, int NTP, int TT, class SZF, class SZI, int NTQ, class SXF,
          class SXI, class SYF, class SYI, int NTA = (N * W + pts_per_thread<T, N, W>() - 1) / pts_per_thread<T, N, W>()>
struct FusedPipeline {
  static constexpr size_t lds = (size_t)N * (N + 1) * sizeof(cpx<T>);
  static void pair_fwd(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_pair_fwd<T, N, W, NTA, TT, SZF>), dim3(nb), dim3(NTA), 0, s, a);
  }
  static void plane(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI>), dim3(nb), dim3(NTQ), lds, s,
                       a);
  }
  static void inv_acc(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_inv_acc<T, N, W, NTA, TT, SZI, true>), dim3(nb), dim3(NTA), 0, s, a);
  }
  static void inv_energy(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_inv_acc<T, N, W, NTA, TT, SZI, false>), dim3(nb), dim3(NTA), 0, s, a);
  }
  static hipError_t prepare() {
    return hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  static Variant describe(const char* name) {
    Variant v{};
    v.name = name;
    v.n = N;
    v.prec = sizeof(T) == 8 ? 1 : 0;
    v.brick = W;
    v.tile = TT;
    v.nt_pencil = NTP;
    v.nt_plane = NTQ;
    v.plane_mode = 0;
    v.rows_per_wg = 0;
    fill_radices(v.zf, v.nzf, SZF{});
    fill_radices(v.zi, v.nzi, SZI{});
    fill_radices(v.xf, v.nxf, SXF{});
    fill_radices(v.xi, v.nxi, SXI{});
    fill_radices(v.yf, v.nyf, SYF{});
    fill_radices(v.yi, v.nyi, SYI{});
    v.plane_lds = lds;
    v.pair_fwd = &pair_fwd;
    v.plane = &plane;
    v.inv_acc = &inv_acc;
    v.inv_energy = &inv_energy;
    v.prepare = &prepare;
    return v;
  }
};

template <typename T, int N, int W, int NTP, int TT, class SZF, class SZI, int RW, int NTQ,
          class SXF, class SXI, class SYF, class SYI,
          int NTA = (N * W + pts_per_thread<T, N, W>() - 1) / pts_per_thread<T, N, W>()>
struct SplitPipeline {
  static constexpr size_t lds = (size_t)RW * (N + 1) * sizeof(cpx<T>);
  static void pair_fwd(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_pair_fwd<T, N, W, NTA, TT, SZF>), dim3(nb), dim3(NTA), 0, s, a);
  }
  static void rows_fwd(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_rows<T, N, RW, NTQ, SXF, false>), dim3(nb), dim3(NTQ), lds, s, a);
  }
  static void rows_inv(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_rows<T, N, RW, NTQ, SXI, true>), dim3(nb), dim3(NTQ), lds, s, a);
  }
  static void cols_conv(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_cols_conv<T, N, W, NTP, SYF, SYI>), dim3(nb), dim3(NTP), 0, s, a);
  }
  static void inv_acc(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_inv_acc<T, N, W, NTA, TT, SZI, true>), dim3(nb), dim3(NTA), 0, s, a);
  }
  static void inv_energy(const PassArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_inv_acc<T, N, W, NTA, TT, SZI, false>), dim3(nb), dim3(NTA), 0, s, a);
  }
  static hipError_t prepare() {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_rows<T, N, RW, NTQ, SXF, false>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rows<T, N, RW, NTQ, SXI, true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  static Variant describe(const char* name) {
    Variant v{};
    v.name = name;
    v.n = N;
    v.prec = sizeof(T) == 8 ? 1 : 0;
    v.brick = W;
    v.tile = TT;
    v.nt_pencil = NTP;
    v.nt_plane = NTQ;
    v.plane_mode = 1;
    v.rows_per_wg = RW;
    fill_radices(v.zf, v.nzf, SZF{});
    fill_radices(v.zi, v.nzi, SZI{});
    fill_radices(v.xf, v.nxf, SXF{});
    fill_radices(v.xi, v.nxi, SXI{});
    fill_radices(v.yf, v.nyf, SYF{});
    fill_radices(v.yi, v.nyi, SYI{});
    v.plane_lds = lds;
    v.pair_fwd = &pair_fwd;
    v.rows_fwd = &rows_fwd;
    v.cols_conv = &cols_conv;
    v.rows_inv = &rows_inv;
    v.inv_acc = &inv_acc;
    v.inv_energy = &inv_energy;
    v.prepare = &prepare;
    return v;
  }
};

}  // namespace hfx
