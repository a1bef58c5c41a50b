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

// Stage twiddle tables live in LDS for the whole workgroup: a few hundred
// bytes, copied once.  Read from global memory inside a transform, a twiddle
// load would make the wave wait for every vector memory operation issued
// before it (loads in flight for the next step, stores of the previous one),
// since one in-order counter tracks them all.
template <typename T, class S>
constexpr int tw_slots() {
  return SchedInfo<S>::tw_count() > 0 ? SchedInfo<S>::tw_count() : 1;
}
template <typename T, class S, int NT>
__device__ __forceinline__ void stage_twiddles(TwEntry<T>* dst, const void* src, int tid) {
  const TwEntry<T>* s = static_cast<const TwEntry<T>*>(src);
  for (int i = tid; i < SchedInfo<S>::tw_count(); i += NT) dst[i] = s[i];
}

// Orbital index of tile position p: screened plans (SCR) reorder the
// orbitals; unscreened plans keep the identity and compile without the table.
template <bool SCR>
__device__ __forceinline__ int orb_at(const PassArgs& a, int p) {
  if constexpr (SCR) return a.perm[p];
  return p;
}

// Whether pair (a, b) of a tile is evaluated: inside the blocks, i <= j on a
// tile inside one diagonal block (row a is orbital i0 + a, column b is
// orbital j0 + b = i0 + joff + b), and, in screened plans, kept by the tile's
// mask (8-orbital column tiles).  Unscreened plans compile without the mask
// tests.
template <int TT, bool SCR>
__device__ __forceinline__ bool pair_live(const TileDesc& td, int ia, int b) {
  if (b >= td.nJ || (td.diag && b + td.joff < ia)) return false;
  if constexpr (SCR && TT == 8) return (keep_word(td, ia >> 3) >> (8 * (ia & 7) + b)) & 1ull;
  return true;
}

// Screened plans: the rows (bit a) and columns (bit b) of a tile that take
// part in at least one evaluated pair.  The others are neither loaded nor
// updated (their products and K psi contributions are all zero).
template <int TT, bool SCR>
__device__ __forceinline__ unsigned live_rows(const TileDesc& td) {
  if constexpr (SCR && TT == 8) {
    unsigned r = 0;
#pragma unroll
    for (int a = 0; a < kMaxRows; ++a)
      r |= (((keep_word(td, a >> 3) >> (8 * (a & 7))) & 0xffull) != 0 ? 1u : 0u) << a;
    return r;
  }
  return ~0u;
}
template <int TT, bool SCR>
__device__ __forceinline__ unsigned live_cols(const TileDesc& td) {
  if constexpr (SCR && TT == 8) {
    unsigned long long k = td.keep0 | td.keep1 | td.keep2 | td.keep3;
    k |= k >> 32;
    k |= k >> 16;
    k |= k >> 8;
    return (unsigned)(k & 0xffull);
  }
  return ~0u;
}
// Next row after ia with an evaluated pair (nI when none is left).
template <bool SCR>
__device__ __forceinline__ int next_live_row(unsigned rows, int ia, int nI) {
  if constexpr (SCR) {
    const unsigned rem = ia + 1 < 32 ? rows >> (ia + 1) : 0u;
    return rem ? ia + 1 + __builtin_ctz(rem) : nI;
  }
  return ia + 1;
}

// scale * (pair-density mean) for the kMaxRows x TT pairs of a tile, [a][b],
// zero outside the tile or without means (float64 plans): staged in LDS so
// that the loops below issue no global loads besides their own data.
template <typename T, int TT, int NT, bool SCR>
__device__ __forceinline__ void stage_means(T* dst, const PassArgs& a, const TileDesc& td,
                                            double scale, int tid) {
  for (int q = tid; q < kMaxRows * TT; q += NT) {
    const int ia = q / TT, b = q - ia * TT;
    dst[q] = (a.mean && ia < td.nI && b < td.nJ)
                 ? (T)(scale * a.mean[(long long)orb_at<SCR>(a, td.i0 + ia) * a.n_orb +
                                      orb_at<SCR>(a, td.j0 + b)])
                 : T(0);
  }
}

// Radix schedules of the half-length forward z transform (length L = NZ / 2)
// of band-limited plans; void where none is compiled.  At 60 the 12 x 5 split
// keeps every thread of a 256-thread workgroup busy in both stages (4 x 15
// leaves half of them idle in the radix-15 stage: 103.6 against 93.5 ms per
// K psi pass at 120^3 / 384 orbitals; 5 x 12 97.7, 6 x 10 95.9).
// Row stride (elements) of the reduced plane input that pass 1 hands to the
// plane pass: half-height planes (HY) hold N / 2 rows of N points, with
// half-width (XD) rows of N / 2 points; the stride is rounded up to 16
// elements, so every 16-column brick row of pass 1 is one whole 128-byte line
// (at 108 or 120 points a row of 54, 60 or 108 elements would leave most
// brick rows straddling two lines).  Full planes keep stride N.
template <int N, bool HY, bool XD>
constexpr int reduced_row_stride() {
  return HY ? ((XD ? N / 2 : N) + 15) / 16 * 16 : N;
}

template <int L> struct HalfZ { using type = void; };
template <> struct HalfZ<24> { using type = Sched<4, 6>; };
template <> struct HalfZ<32> { using type = Sched<4, 8>; };
template <> struct HalfZ<36> { using type = Sched<4, 9>; };
template <> struct HalfZ<40> { using type = Sched<4, 10>; };
template <> struct HalfZ<48> { using type = Sched<4, 12>; };
template <> struct HalfZ<54> { using type = Sched<6, 9>; };
template <> struct HalfZ<60> { using type = Sched<12, 5>; };
template <> struct HalfZ<64> { using type = Sched<8, 8>; };

// ---------------------------------------------------------------------------
// Pass 1: pair product + forward z FFT on bricks.
// On full planes a brick is W consecutive points of the xy plane in storage
// order (W x values of one row where N is a multiple of W; at other N a brick
// may run on into the next row), so every brick row of psi and of the grids
// is whole 64- or 128-byte segments, and no brick is partly off the grid.
// Two pair grids are transformed together: LDS holds [z][2W] with the brick
// of grid g in columns [gW, gW + W).  Thread tid forms the products at brick
// points p = tid + k NT (k < PT, contiguous x for coalesced psi reads) for both
// grids; the transform starts from LDS and its last stage stores straight to
// HBM.  psi of the tile's J block stays in registers for the whole tile.
// With PIL the I block is loaded once too, into LDS (each thread reads back
// only what it wrote), so the loop over orbitals issues no global loads: its
// HBM stores are never waited for (one in-order counter tracks loads and
// stores, so a later load would wait for them).  Without PIL, psi_a is loaded
// per orbital.
// N: grid points along x and y; NZ: along z (slab cells: NZ != N).
// HZ (band-limited plans with 2 kz_max + 1 <= NZ / 2): the pair densities,
// whose z spectrum lies in |kz| <= kz_max, are sampled exactly by the even z
// points, so the forward z transform runs at length NZ / 2 on those (half the
// orbital reads and half the transform work).  For such data the half-length
// sum over even points is half the full-length sum at every kept frequency;
// the products are doubled (exact) and half-length frequency k maps to grid
// plane k (k <= kz_max) or k + NZ / 2 (k >= NZ / 2 - kz_max).
// HY (plans whose plane pass takes half-height input): bricks run at the even
// rows y = 2y' only and store row y' of their planes, with doubled products
// (rows of reduced_row_stride elements at the plane's start).
// XD (with HY, half-width input too): the W columns of a brick are the even
// x = 2x' (psi read over 2W columns), stored as column x' of rows of N / 2
// points (a quarter plane).
template <typename T, int N, int W, int NT, int TT, class SZF, bool PIL, bool SCR, int NZ = N,
          bool HZ = false, class SZH = typename HalfZ<NZ / 2>::type, bool HY = false,
          bool XD = false>
__global__ void __launch_bounds__(NT) k_pair_fwd(PassGroup grp) {
  int sys_ = 0;
  const int lg_ = grp.locate(xcd_remap(blockIdx.x, gridDim.x), sys_);
  const PassArgs& a = grp.a[sys_];
  static_assert(TT % 4 == 0, "tile must hold whole grid pairs");
  constexpr int W2 = 2 * W;
  constexpr int ZL = HZ ? NZ / 2 : NZ;  // transform length
  using SZ = std::conditional_t<HZ, SZH, SZF>;
  using G = Geom<T, ZL, W2, NT, true, W2, 1>;
  using L = LastStage<G, SZ>;
  using E = FFT<G, false, SZ>;
  constexpr int RL = SchedInfo<SZ>::last;
  static_assert(!XD || HY, "half-width input comes with half-height input");
  constexpr int NXI = XD ? N / 2 : N;          // x points (columns) stored per row
  constexpr int XST = reduced_row_stride<N, HY, XD>();  // stored row stride
  static_assert(!HY || (N / 2) * XST <= N * N, "reduced planes fit the plane's slot");
  constexpr int NXB = (NXI + W - 1) / W;
  // full planes: a brick is W consecutive points of the xy plane in storage
  // order (flat bricks, whole cache lines at any N); reduced planes: W
  // columns of one stored row
  static_assert(HY || (N * N) % W == 0, "flat bricks tile the plane");
  constexpr int BR = HY ? (N / 2) * NXB : N * N / W;  // bricks per tile pair
  constexpr int LIM = HY ? NXI : N * N;  // bound of x0 + m
  constexpr int P = ZL * W;
  constexpr int PT = (P + NT - 1) / NT;
  constexpr long long NR = (long long)NZ * N * N;
  constexpr int ZSL = (ZL / RL) * N * N;  // offset between legs of a last-stage butterfly
  constexpr int ZS = HZ ? 2 : 1;         // z stride of the product points
  constexpr int YS = HY ? 2 : 1;         // y stride of the brick rows
  constexpr int XS = XD ? 2 : 1;         // x stride of the brick columns
  __shared__ cpx<T> lds[ZL * W2];
  __shared__ TwEntry<T> twl[tw_slots<T, SZ>()];
  __shared__ T mul[kMaxRows * TT];  // pair-density means of the tile, [a][b]
  __shared__ T pil[PIL ? TT * PT * NT : 1];  // psi of the I block, [a][k][tid]
  const int tid = threadIdx.x;
  const int lg = lg_;
  const int t = lg / BR, br = lg - t * BR;
  // y: the stored row (read at YS y); flat bricks: y = 0, x0 = flat offset
  const int y = HY ? br / NXB : 0, x0 = HY ? (br - y * NXB) * W : br * W;
  const TileDesc td = a.tiles[t];
  const T* __restrict__ psi = static_cast<const T*>(a.psi);
  stage_twiddles<T, SZ, NT>(twl, HZ ? a.tw_zh : a.tw_zf, tid);
  stage_means<T, TT, NT, SCR>(mul, a, td, 1.0, tid);
  const TwEntry<T>* tw = twl;
  cpx<T>* __restrict__ grids = static_cast<cpx<T>*>(a.grids);

  int offA[PT], ldsA[PT];
  bool vA[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int p = tid + k * NT;
    const int z = p / W, m = p - (p / W) * W;
    vA[k] = p < P && (x0 + m) < LIM;
    offA[k] = vA[k] ? (ZS * z * N + YS * y) * N + XS * (x0 + m) : 0;
    ldsA[k] = z * W2 + m;
  }
  int offL[L::PER], gL[L::PER];
  bool vL[L::PER];
  unsigned kzL[L::PER];  // bit r: leg r (frequency j + r ZL / RL) lies on a kept kz plane
  unsigned hiL[L::PER];  // HZ, bit r: leg r is a negative frequency (grid plane + NZ / 2)
#pragma unroll
  for (int i = 0; i < L::PER; ++i) {
    int m = 0, j = 0;
    L::mj(tid, i, m, j);
    gL[i] = m / W;
    const int mx = m - gL[i] * W;
    vL[i] = L::valid(tid, i) && (x0 + mx) < LIM;
    offL[i] = vL[i] ? j * N * N + y * XST + x0 + mx : 0;
    kzL[i] = 0;
    hiL[i] = 0;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int k = j + r * (ZL / RL);
      kzL[i] |= (kz_kept(k, ZL, a.kz_max) ? 1u : 0u) << r;
      if constexpr (HZ) hiL[i] |= (2 * k >= ZL ? 1u : 0u) << r;
    }
  }

  // psi of the J block (registers) and, with PIL, of the I block (LDS),
  // zero off the grid; loads issued four orbitals at a time before any use
  T pj[TT][PT];
  const unsigned cols = live_cols<TT, SCR>(td), rows = live_rows<TT, SCR>(td);
  static_for<0, TT / 4>([&](auto hc) {
    constexpr int b0 = 4 * decltype(hc)::value;
    T xj[4][PT], xi[PIL ? 4 : 1][PT];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T* pb = psi + (long long)orb_at<SCR>(a, td.j0 + (b0 + q < td.nJ ? b0 + q : 0)) * NR;
      if constexpr (SCR) {
        // columns without an evaluated pair are not read
        const bool live = (cols >> (b0 + q)) & 1u;
#pragma unroll
        for (int k = 0; k < PT; ++k) xj[q][k] = live ? pb[offA[k]] : T(0);
      } else {
#pragma unroll
        for (int k = 0; k < PT; ++k) xj[q][k] = pb[offA[k]];
      }
      if constexpr (PIL) {
        const T* pa = psi + (long long)orb_at<SCR>(a, td.i0 + (b0 + q < td.nI ? b0 + q : 0)) * NR;
#pragma unroll
        for (int k = 0; k < PT; ++k) xi[q][k] = pa[offA[k]];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < PT; ++k) {
        pj[b0 + q][k] = (b0 + q < td.nJ && vA[k]) ? xj[q][k] : T(0);
        if constexpr (PIL)
          pil[((b0 + q) * PT + k) * NT + tid] = (b0 + q < td.nI && vA[k]) ? xi[PIL ? q : 0][k] : T(0);
      }
  });
  __syncthreads();

  for (int ia = 0; ia < td.nI; ++ia) {
    if constexpr (SCR) {
      if (!((rows >> ia) & 1u)) continue;  // no evaluated pair in this row
    }
    T pa[PT];
    if constexpr (PIL) {
#pragma unroll
      for (int k = 0; k < PT; ++k) pa[k] = pil[(ia * PT + k) * NT + tid];
    } else {
      const T* pa_ptr = psi + (long long)orb_at<SCR>(a, td.i0 + ia) * NR;
#pragma unroll
      for (int k = 0; k < PT; ++k) pa[k] = vA[k] ? pa_ptr[offA[k]] : T(0);
    }
    static_for<0, TT / 4>([&](auto bq) {
      constexpr int b0 = 4 * decltype(bq)::value;  // pairs (a, b0 .. b0 + 3), grids 2bq, 2bq+1
      // grid g carries pairs (a, b0 + 2g) and (a, b0 + 2g + 1)
      const bool use0 = pair_live<TT, SCR>(td, ia, b0) || pair_live<TT, SCR>(td, ia, b0 + 1);
      const bool use1 = pair_live<TT, SCR>(td, ia, b0 + 2) || pair_live<TT, SCR>(td, ia, b0 + 3);
      if (!use0 && !use1) return;
      // pair-density means (float32 plans): transforms see zero-mean densities
      T mu[4], on[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        mu[q] = mul[ia * TT + b0 + q];
        // pairs not evaluated (screened, or below the diagonal) transform as
        // zeros, so they add no rounding to the pair sharing their grid; the
        // half-length transform takes doubled products
        on[q] = pair_live<TT, SCR>(td, ia, b0 + q) ? T(ZS * YS * XS) : T(0);
      }
#pragma unroll
      for (int k = 0; k < PT; ++k)
        if (tid + k * NT < P) {
          const T in = vA[k] ? T(1) : T(0);  // columns beyond the grid stay zero
          lds[ldsA[k]] = {on[0] * (pa[k] * pj[b0][k] - in * mu[0]),
                          on[1] * (pa[k] * pj[b0 + 1][k] - in * mu[1])};
          lds[ldsA[k] + W] = {on[2] * (pa[k] * pj[b0 + 2][k] - in * mu[2]),
                              on[3] * (pa[k] * pj[b0 + 3][k] - in * mu[3])};
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
          for (int r = 0; r < RL; ++r)
            if ((kzL[i] >> r) & 1u)
              g[offL[i] + r * ZSL + (((hiL[i] >> r) & 1u) ? (NZ / 2) * N * N : 0)] =
                  out[i * RL + r];
        }
      }
    });
  }
}

// ---------------------------------------------------------------------------
// Pass 3: inverse z FFT + pair energies + K psi accumulation on bricks (flat
// bricks, as in pass 1).
// Two pair grids are transformed together ([z][2W] in LDS, as in pass 1).
// The inverse transform leaves the potentials in LDS in natural order; the
// accumulation then uses its own point map: thread tid owns brick points
// p = tid + k NT (k < PT), contiguous x for coalesced K psi traffic.  The
// J-side accumulators stay in registers for the whole tile; psi of the J
// block stays in registers too, or (PJL) in LDS, where each thread reads
// back only the points it wrote (no barrier needed).  The pair energy of a
// thread's points is summed in the working precision per pair and added to a
// float64 accumulator once per pair.
//
// Latency hiding: the old K psi values of orbital a are loaded with its psi,
// so the update at the end of the orbital is a plain store.  With PF, while
// one grid pair is transformed the loads of the next one are in flight
// (second register buffer), and the next orbital's psi and old K psi values
// are loaded one step ahead.
// KZ: band-limited plans (PassArgs::kz_max < NZ / 2) do not load the pruned
// kz planes; other plans (KZ = 0) compile without the plane tests.  KZ = 1
// (most planes kept): pruned legs load zeros from the plan's zero block, so
// every load stays unconditional; KZ = 2 (many planes pruned): pruned legs are
// not loaded at all (the compiler branches around them, and whole waves skip
// the legs of fully pruned frequency blocks).
// FL (flat loads, with PF): a grid pair's brick is loaded by all threads in
// its natural [z][2W] order (neighbouring threads on neighbouring x), a few
// elements each, and written to LDS before the transform, which then starts
// from LDS.  The prefetch of the next grid pair then holds NZ * 2W / NT values
// per thread instead of the first stage's legs, which for large radices sit
// in a quarter of the threads (a radix-16 first stage over 32 columns of 128
// points is 256 butterflies) and cost 16 complex registers each.
template <typename T, int N, int W, int NT, int TT, class SZI, bool ACC, bool PJL, bool PF,
          bool SCR, int NZ = N, int KZ = 0, bool FL = false, int NG = 2>
__global__ void __launch_bounds__(NT)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) k_inv_acc(PassGroup grp) {
  int sys_ = 0;
  const int lg_ = grp.locate(xcd_remap(blockIdx.x, gridDim.x), sys_);
  const PassArgs& a = grp.a[sys_];
  static_assert(TT % (2 * NG) == 0, "a row of the tile must hold whole transforms");
  static_assert(NG == 2 || FL, "four grids per transform come with flat loads");
  constexpr int W2 = NG * W;               // columns of one transform (NG grids)
  constexpr int QB = TT / (2 * NG);        // transforms per orbital a
  using G = Geom<T, NZ, W2, NT, true, W2, 1>;
  using F = FirstStage<G, SZI>;
  using E = FFT<G, true, SZI>;
  constexpr int RF = SchedInfo<SZI>::first;
  // flat bricks: W consecutive points of the xy plane in storage order
  static_assert((N * N) % W == 0, "flat bricks tile the plane");
  constexpr int BR = N * N / W;
  constexpr int P = NZ * W;                // brick points
  constexpr int PT = (P + NT - 1) / NT;    // accumulation points per thread
  constexpr long long NR = (long long)NZ * N * N;
  constexpr int ZSF = (NZ / RF) * N * N;   // offset between legs of a first-stage butterfly
  __shared__ cpx<T> lds[NZ * W2];
  __shared__ double red[pow2_at_least<NT>()];
  __shared__ T pjl[PJL ? TT * PT * NT : 1];  // [b][k][tid]
  __shared__ TwEntry<T> twl[tw_slots<T, SZI>()];
  __shared__ T dcl[kMaxRows * TT];  // v(0) * pair-density mean, [a][b]
  const int tid = threadIdx.x;
  const int lg = lg_;
  const int t = lg / BR, br = lg - t * BR;
  const int x0 = br * W;  // flat offset of the brick in the xy plane
  constexpr int LIM = N * N;
  const TileDesc td = a.tiles[t];
  const T* __restrict__ psi = static_cast<const T*>(a.psi);
  T* __restrict__ kpsi = static_cast<T*>(a.kpsi);
  stage_twiddles<T, SZI, NT>(twl, a.tw_zi, tid);
  stage_means<T, TT, NT, SCR>(dcl, a, td, a.v0, tid);
  __syncthreads();
  const TwEntry<T>* tw = twl;
  const cpx<T>* __restrict__ grids = static_cast<const cpx<T>*>(a.grids);

  int offF[F::PER], gF[F::PER];
  bool vF[F::PER];
  unsigned kzF[F::PER];  // bit r: leg r (frequency j + r NZ / RF) lies on a kept kz plane
#pragma unroll
  for (int i = 0; i < F::PER; ++i) {
    int m = 0, j = 0;
    F::mj(tid, i, m, j);
    gF[i] = m / W;
    const int mx = m - gF[i] * W;
    vF[i] = F::valid(tid, i) && (x0 + mx) < LIM;
    offF[i] = vF[i] ? j * N * N + x0 + mx : 0;
    kzF[i] = ~0u;
    if constexpr (KZ != 0) {
      kzF[i] = 0;
#pragma unroll
      for (int r = 0; r < RF; ++r) kzF[i] |= (kz_kept(j + r * (NZ / RF), NZ, a.kz_max) ? 1u : 0u) << r;
    }
  }
  int offA[PT], ldsA[PT];
  bool vA[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int p = tid + k * NT;
    const int z = p / W, m = p - (p / W) * W;
    vA[k] = p < P && (x0 + m) < LIM;
    offA[k] = vA[k] ? z * N * N + x0 + m : 0;
    ldsA[k] = z * W2 + m;
  }

  // FL: element e = tid + k NT of the brick, e = z NG W + c (c: column of
  // the transform, grid c / W, flat point x0 + c mod W) -- the LDS index of the engine
  constexpr int FE = NZ * W2;
  constexpr int FLV = FL ? (FE + NT - 1) / NT : 1;
  int offFL[FLV], gFL[FLV];
  bool vFL[FLV], kzFL[FLV];
#pragma unroll
  for (int k = 0; k < FLV; ++k) {
    const int e = tid + k * NT;
    const int z = e / W2, c = e - (e / W2) * W2;
    const int g = c / W, m = c - (c / W) * W;
    vFL[k] = FL && e < FE && x0 + m < LIM;
    gFL[k] = g;
    offFL[k] = vFL[k] ? z * N * N + x0 + m : 0;
    kzFL[k] = KZ == 0 || kz_kept(z < NZ ? z : 0, NZ, a.kz_max);
  }

  T pjr[PJL ? 1 : TT][PT];
  auto pj = [&](int b, int k) -> T { return PJL ? pjl[(b * PT + k) * NT + tid] : pjr[PJL ? 0 : b][k]; };
  T accJ[ACC ? TT : 1][PT];
  const unsigned cols = live_cols<TT, SCR>(td), rows = live_rows<TT, SCR>(td);
  // psi of the J block (zero off the grid); for LDS, four orbitals at a time,
  // all loads before the stores
  static_for<0, TT / 4>([&](auto hc) {
    constexpr int b0 = 4 * decltype(hc)::value;
    T x[4][PT];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool bv = b0 + q < td.nJ;
      const T* pb = psi + (long long)orb_at<SCR>(a, td.j0 + (bv ? b0 + q : 0)) * NR;
      if constexpr (SCR) {
        const bool live = (cols >> (b0 + q)) & 1u;
#pragma unroll
        for (int k = 0; k < PT; ++k) x[q][k] = live ? pb[offA[k]] : T(0);
      } else {
#pragma unroll
        for (int k = 0; k < PT; ++k) x[q][k] = pb[offA[k]];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool bv = b0 + q < td.nJ;
#pragma unroll
      for (int k = 0; k < PT; ++k) {
        const T v = (bv && vA[k]) ? x[q][k] : T(0);
        if constexpr (PJL) pjl[((b0 + q) * PT + k) * NT + tid] = v;
        else pjr[PJL ? 0 : b0 + q][k] = v;
      }
    }
  });
#pragma unroll
  for (int b = 0; b < (ACC ? TT : 1); ++b)
#pragma unroll
    for (int k = 0; k < PT; ++k) accJ[b][k] = T(0);
  double eacc = 0.0;
  T pa[PT], acca[PT], kold[ACC ? PT : 1];
  T pa_n[PF ? PT : 1], kold_n[(PF && ACC) ? PT : 1];

  // transform bq of orbital a carries pairs (a, 2 NG bq .. 2 NG bq + 2 NG - 1);
  // bit g of the mask: grid g (pairs b0 + 2g, b0 + 2g + 1) has an evaluated pair
  auto uses = [&](int ia, int bq) {
    const int b0 = 2 * NG * bq;
    unsigned um = 0;
#pragma unroll
    for (int g = 0; g < NG; ++g)
      um |= (pair_live<TT, SCR>(td, ia, b0 + 2 * g) || pair_live<TT, SCR>(td, ia, b0 + 2 * g + 1)
                 ? 1u : 0u) << g;
    return um;
  };
  // Loads below are issued unconditionally: masked-off lanes read a valid
  // dummy address (data written earlier in the batch: finite), and legs on
  // pruned kz planes (never written) read zeros from the plan's zero block.
  // With no branches after them, the compiler counts the loads in flight and
  // waits only for the ones needed.  Dummy values are harmless: a
  // grid of an unused pair is transformed but its potentials are never used,
  // and at points outside the grid psi_b = 0 (set at the tile load), so
  // energies and K psi_a get exact zeros there, while K psi_b is not stored
  // there.
  auto load_pair = [&](int ia, int bq, cpx<T>* v) {
    const unsigned um = uses(ia, bq);
    const int slot0 = td.slot0 + ia * (TT / 2) + NG * bq;
#pragma unroll
    for (int i = 0; i < F::PER; ++i) {
      const bool ok = vF[i] && ((um >> gF[i]) & 1u);
      const cpx<T>* dummy = grids + (long long)td.slot0 * NR;
      const cpx<T>* g = ok ? grids + (long long)(slot0 + gF[i]) * NR + offF[i] : dummy;
      if constexpr (KZ == 1) {
        // a leg on a pruned plane loads from the plan's zero block: every
        // load is issued and its value used as loaded (no branch, no select).
        // All lanes read the block's first element (one request per wave),
        // so no per-lane pointer stays live across the loop: at 96^3 a
        // per-lane one cost three spilled registers in the loop, whose
        // scratch lines were evicted by the grid stream and written back
        // (about 10 % extra HBM traffic)
        const cpx<T>* zero = static_cast<const cpx<T>*>(a.zero);
#pragma unroll
        for (int r = 0; r < RF; ++r) {
          const bool kept = (kzF[i] >> r) & 1u;
          v[i * RF + r] = *(kept ? g + (ok ? r * ZSF : 0) : zero);
        }
      } else if constexpr (KZ == 2) {
        // the value of a pruned leg is discarded, so its load is skipped
#pragma unroll
        for (int r = 0; r < RF; ++r) {
          const bool kept = (kzF[i] >> r) & 1u;
          const cpx<T> val = *(ok && kept ? g + r * ZSF : dummy);
          v[i * RF + r] = kept ? val : cpx<T>{T(0), T(0)};
        }
      } else {
#pragma unroll
        for (int r = 0; r < RF; ++r) v[i * RF + r] = g[ok ? r * ZSF : 0];
      }
    }
  };
  // FL: the grid pair's brick in flat order (same dummy and zero-block rules)
  auto load_flat = [&](int ia, int bq, cpx<T>* v) {
    const unsigned um = uses(ia, bq);
    const int slot0 = td.slot0 + ia * (TT / 2) + NG * bq;
    const cpx<T>* dummy = grids + (long long)td.slot0 * NR;
#pragma unroll
    for (int k = 0; k < FLV; ++k) {
      const bool ok = vFL[k] && ((um >> gFL[k]) & 1u);
      const cpx<T>* g = ok ? grids + (long long)(slot0 + gFL[k]) * NR + offFL[k] : dummy;
      if constexpr (KZ == 1) {
        const cpx<T>* zero = static_cast<const cpx<T>*>(a.zero);
        v[k] = *(kzFL[k] ? g : zero);
      } else if constexpr (KZ == 2) {
        const cpx<T> val = *(ok && kzFL[k] ? g : dummy);
        v[k] = kzFL[k] ? val : cpx<T>{T(0), T(0)};
      } else {
        v[k] = *g;
      }
    }
  };
  // psi and old K psi of orbital a at the thread's points (offA = 0 off the grid)
  auto load_orbital = [&](int ia, T* p, T* ko) {
    const int oa = orb_at<SCR>(a, td.i0 + ia);
    const T* pa_ptr = psi + (long long)oa * NR;
    const T* ka = kpsi + (long long)oa * NR;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      p[k] = pa_ptr[offA[k]];
      if constexpr (ACC) ko[k] = ka[offA[k]];
    }
  };
  // inverse transform of the grid pair in v, then energies and K psi updates
  auto process = [&](auto bqc, int ia, cpx<T>* v) {
    constexpr int b0 = 2 * NG * decltype(bqc)::value;
    const unsigned um = uses(ia, decltype(bqc)::value);
    if (!um) return;
    {
      cpx<T> out[LastStage<G, SZI>::VALS];
      if constexpr (FL) {
#pragma unroll
        for (int k = 0; k < FLV; ++k)
          if (FE % NT == 0 || tid + k * NT < FE) lds[tid + k * NT] = v[k];
        __syncthreads();
        E::lds2reg(lds, tw, tid, out);
      } else {
        E::reg2reg(v, lds, tw, tid, out);
      }
      E::store_last(out, lds, tid);
    }
    __syncthreads();
    // one grid's potentials at a time (bounded registers)
    cpx<T> pot[PT];
    static_for<0, 2 * NG>([&](auto q) {
      constexpr int gq = decltype(q)::value / 2, half = decltype(q)::value % 2;
      constexpr int b = b0 + decltype(q)::value;
      if constexpr (half == 0) {
#pragma unroll
        for (int k = 0; k < PT; ++k)
          pot[k] = tid + k * NT < P ? lds[ldsA[k] + gq * W] : cpx<T>{T(0), T(0)};
      }
      if (b >= td.nJ) return;
      if (!((um >> gq) & 1u)) return;
      // weight of e_ab in sum_{i,j} e_ij: 2 for a != b, 1 for a == b, 0 for
      // pairs not evaluated
      if (!pair_live<TT, SCR>(td, ia, b)) return;
      const int w = (td.diag && b + td.joff == ia) ? 1 : 2;
      // G = 0 part of v_ab when the mean was taken out of the transform;
      // its energy v0 * Omega * mu_ab^2 is added in float64 at the reduction
      const T dc = dcl[ia * TT + b];
      T es = T(0);
#pragma unroll
      for (int k = 0; k < PT; ++k) {
        const T vz = half ? pot[k].im : pot[k].re;  // zero-mean part
        const T pjb = pj(b, k);
        es += vz * pjb * pa[k];                     // rho_ab v_ab
        if constexpr (ACC) {
          const T vv = vz + dc;
          accJ[b][k] -= vv * pa[k];
          if (w == 2) acca[k] -= vv * pjb;
        }
      }
      eacc += (double)w * (double)es;
    });
    __syncthreads();  // LDS is rewritten by the next transform
  };

  auto store_orbital = [&](int ia) {
    if constexpr (ACC) {
      T* ka = kpsi + (long long)orb_at<SCR>(a, td.i0 + ia) * NR;
#pragma unroll
      for (int k = 0; k < PT; ++k)
        if (vA[k]) ka[offA[k]] = kold[k] + acca[k];
    }
  };
  if constexpr (PF) {
    constexpr int PV = FL ? FLV : F::VALS;
    cpx<T> vc[PV], vn[PV];
    auto load_next = [&](int ia, int bq, cpx<T>* v) {
      if constexpr (FL) load_flat(ia, bq, v);
      else load_pair(ia, bq, v);
    };
    const int ia0 = next_live_row<SCR>(rows, -1, td.nI);
    if (ia0 < td.nI) {
      load_orbital(ia0, pa, kold);
      load_next(ia0, 0, vc);
    }
    for (int ia = ia0; ia < td.nI;) {
      const int nx = next_live_row<SCR>(rows, ia, td.nI);
#pragma unroll
      for (int k = 0; k < PT; ++k) acca[k] = T(0);
      static_for<0, QB>([&](auto bq) {
        constexpr int q = decltype(bq)::value;
        // next step's loads go out before this step's transform
        if constexpr (q + 1 < QB) {
          load_next(ia, q + 1, vn);
        } else if (nx < td.nI) {
          load_orbital(nx, pa_n, kold_n);
          load_next(nx, 0, vn);
        }
        process(bq, ia, vc);
#pragma unroll
        for (int e = 0; e < PV; ++e) vc[e] = vn[e];
      });
      store_orbital(ia);
#pragma unroll
      for (int k = 0; k < PT; ++k) {
        pa[k] = pa_n[k];
        if constexpr (ACC) kold[k] = kold_n[k];
      }
      ia = nx;
    }
  } else {
    static_assert(!FL, "flat loads are a form of the prefetching loop");
    for (int ia = next_live_row<SCR>(rows, -1, td.nI); ia < td.nI;
         ia = next_live_row<SCR>(rows, ia, td.nI)) {
      load_orbital(ia, pa, kold);
#pragma unroll
      for (int k = 0; k < PT; ++k) acca[k] = T(0);
      static_for<0, QB>([&](auto bq) {
        if (!uses(ia, decltype(bq)::value)) return;
        cpx<T> v[F::VALS];
        load_pair(ia, decltype(bq)::value, v);
        process(bq, ia, v);
      });
      store_orbital(ia);
    }
  }
  if constexpr (ACC) {
    // four orbitals at a time: all old values first (one wait), then the stores
    static_for<0, TT / 4>([&](auto hc) {
      constexpr int b0 = 4 * decltype(hc)::value;
      T old[4][PT];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool bv = b0 + q < td.nJ;
        const T* kb = kpsi + (long long)orb_at<SCR>(a, td.j0 + (bv ? b0 + q : 0)) * NR;
        if constexpr (SCR) {
          // columns without an evaluated pair keep their K psi untouched
          const bool live = (cols >> (b0 + q)) & 1u;
#pragma unroll
          for (int k = 0; k < PT; ++k) old[q][k] = live ? kb[offA[k]] : T(0);
        } else {
#pragma unroll
          for (int k = 0; k < PT; ++k) old[q][k] = kb[offA[k]];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T* kb = kpsi + (long long)orb_at<SCR>(a, td.j0 + (b0 + q < td.nJ ? b0 + q : 0)) * NR;
        const bool live = !SCR || ((cols >> (b0 + q)) & 1u);
#pragma unroll
        for (int k = 0; k < PT; ++k)
          if (live && b0 + q < td.nJ && vA[k]) kb[offA[k]] = old[q][k] + accJ[b0 + q][k];
      }
    });
  }
  const double s = block_sum<NT>(eacc, red);
  if (tid == 0) a.partials[a.part_base + lg] = s;
}

// ---------------------------------------------------------------------------
// Pass 2: fused plane convolution for one kz plane of one pair grid.
// Waves per SIMD that the plane's LDS allows (planes per compute unit x
// wavefronts per plane / 4 SIMDs): register use is capped so that registers
// never admit fewer planes than LDS does.
template <typename T, int N, int NT>
constexpr int plane_waves_per_eu() {
  constexpr int lds = N * (N + 1) * (int)sizeof(cpx<T>) + 4096;  // plane + twiddle tables
  constexpr int planes = (160 * 1024) / lds > 0 ? (160 * 1024) / lds : 1;
  constexpr int w = (planes * ((NT + 63) / 64) + 3) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// The v(G) factors of a plane are loaded into registers when the plane starts
// (after its rows), so the multiply between the y transforms never waits for
// them: a load issued behind the barriers of the forward transforms would
// stall every wave of the workgroup at once.
// PP (persistent, prefetching): for planes that leave room for one plane per
// compute unit, a workgroup per compute unit walks the planes of the launch
// (L, L + grid, ...) with the twiddles staged once, and issues the HBM loads
// of its next plane's rows as soon as the forward x transform of the current
// one has consumed its input registers, so they are in flight during the y
// transforms, the multiply and the inverse x transform.  The v(G) loads of a
// plane are issued before that prefetch, so waiting for them never waits for
// it (one in-order counter tracks the loads).
// QB > 0 (band-limited plans whose pair densities vanish for |kx| > QB):
// the forward x transform stores zeros in the columns beyond the band and
// the y transforms, the multiply and the inverse y transforms run on the
// 2 QB + 1 columns of the band only (a band geometry of the engine); the
// inverse x transforms read the zeros.
// GM (grid-major plane order): logical plane L is plane L mod kp of grid
// L / kp (kp kept planes per grid), so workgroups running together stream
// neighbouring planes of one grid; kz-major order (GM false) has them read the
// same plane of many grids, whose addresses coincide modulo the grid size.
// HY (band-limited along y too, 2 ky_max + 1 <= N / 2; with QB): pass 1 has
// stored only the even rows y = 2y' (row y' of the plane, products doubled),
// which sample the plane's y band exactly.  The forward x transforms run on
// those N / 2 rows, the forward y transforms at length N / 2 (schedule SYH),
// and the multiplied spectrum is written to its full-length rows (half-length
// frequency k: row k below N / 4, else k + N / 2; the rows between, zeros)
// before the inverse y transforms of length N, which restore every row.
// In both modes the input rows lie reduced_row_stride elements apart.
// XD (with HY, band-limited along x too): the input rows hold the even
// x = 2x' only (N / 2 points each, a quarter plane); the forward x transforms
// run at length N / 2 (the same half-length schedule) and place half-length
// frequency k in column k below N / 4, else k + N / 2; the inverse x
// transforms read the band's columns and take zeros elsewhere.
template <typename T, int N, int NT, class SXF, class SXI, class SYF, class SYI, bool SW = false,
          bool PP = false, int NZ = N, int QB = 0, bool GM = false, bool HY = false,
          class SYH = SYF, bool XD = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(plane_waves_per_eu<T, N, NT>())))
k_plane_conv(PassGroup grp) {
  int sys_ = 0;
  const int lg_ = grp.locate(xcd_remap(blockIdx.x, gridDim.x), sys_);
  const PassArgs& a = grp.a[sys_];
  static_assert(!SW || N % 8 == 0, "swizzle needs whole blocks of 8");
  static_assert(QB == 0 || (!SW && 2 * QB + 1 < N), "band columns: no swizzle, inside the row");
  static_assert(!HY || (QB > 0 && N % 4 == 0), "half-height planes come with band columns");
  static_assert(!XD || (HY && QB == N / 4), "half-width input comes with half-height input");
  constexpr int P = N + 1;
  constexpr int NI = HY ? N / 2 : N;  // rows of the plane's input
  constexpr int NXI = XD ? N / 2 : N;  // points per input row
  constexpr int XST = reduced_row_stride<N, HY, XD>();  // input row stride
  constexpr int MB = QB ? 2 * QB + 1 : N;
  using GX = Geom<T, N, N, NT, false, 1, P, SW ? 1 : 0>;  // rows: sequence m = y, element n = x
  using GXF = Geom<T, NXI, NI, NT, false, 1, P, SW ? 1 : 0>;  // the input rows
  using SXFX = std::conditional_t<XD, SYH, SXF>;
  // columns: sequence m = x (or the m-th column of the band), element n = y
  using GY = Geom<T, N, MB, NT, true, P, 1, SW ? 2 : (QB ? 3 : 0)>;
  using GYF = Geom<T, NI, MB, NT, true, P, 1, SW ? 2 : (QB ? 3 : 0), N>;  // forward y
  using SYFX = std::conditional_t<HY, SYH, SYF>;
  using EXF = FFT<GXF, false, SXFX>;
  using EXI = FFT<GX, true, SXI>;
  using EYF = FFT<GYF, false, SYFX>;
  using EYI = FFT<GY, true, SYI>;
  using FX = FirstStage<GXF, SXFX>;
  using LXF = LastStage<GXF, SXFX>;
  using FXI = FirstStage<GX, SXI>;
  using LY = LastStage<GYF, SYFX>;
  using FYI = FirstStage<GY, SYI>;
  using LYI = LastStage<GY, SYI>;
  using LXI = LastStage<GX, SXI>;
  static_assert(HY || SchedInfo<SYI>::first == SchedInfo<SYF>::last, "fused y schedules");
  static_assert(HY || FYI::VALS == LY::VALS, "fused y register maps");
  constexpr long long NR = (long long)NZ * N * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* plane = reinterpret_cast<cpx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int lg = lg_;
  const int total = a.n_active * kz_planes(NZ, a.kz_max);  // planes of this launch, kz-major
  cpx<T>* __restrict__ gbase = static_cast<cpx<T>*>(a.grids);

  if (lg >= total) return;
  __shared__ TwEntry<T> twxf[tw_slots<T, SXFX>()], twyf[tw_slots<T, SYFX>()],
      twyi[tw_slots<T, SYI>()], twxi[tw_slots<T, SXI>()];
  stage_twiddles<T, SXFX, NT>(twxf, XD ? a.tw_zh : a.tw_xf, tid);  // visible after the first barrier
  // half-height: the half-length schedule is the plan's half-length z one
  stage_twiddles<T, SYFX, NT>(twyf, HY ? a.tw_zh : a.tw_yf, tid);
  stage_twiddles<T, SYI, NT>(twyi, a.tw_yi, tid);
  stage_twiddles<T, SXI, NT>(twxi, a.tw_xi, tid);
  const int kp_ = kz_planes(NZ, a.kz_max);
  auto plane_kz = [&](int L) {
    return kz_of_plane(GM ? L - (L / kp_) * kp_ : L / a.n_active, NZ, a.kz_max);
  };
  auto plane_base = [&](int L) {
    const int ai = GM ? L / kp_ : L - (L / a.n_active) * a.n_active;
    return gbase + (long long)a.active[ai] * NR + (long long)plane_kz(L) * N * N;
  };
  // x-forward stage-0 inputs straight from HBM (rows, x contiguous)
  auto load_rows = [&](const cpx<T>* __restrict__ base, cpx<T>* v, int t) {
#pragma unroll
    for (int i = 0; i < FX::PER; ++i) {
      if (!FX::valid(t, i)) continue;
      int m, j;
      FX::mj(t, i, m, j);
#pragma unroll
      for (int r = 0; r < SchedInfo<SXFX>::first; ++r)
        v[i * SchedInfo<SXFX>::first + r] = base[m * XST + FX::in_pos(j, r)];
    }
  };
  // v(G) / N_r at the thread's multiply points of plane L
  auto load_v = [&](int L, T* f, int t) {
    const T* __restrict__ vt =
        static_cast<const T*>(a.vtab) + (long long)plane_kz(L) * N * N;
#pragma unroll
    for (int i = 0; i < LY::PER; ++i) {
      int m = 0, j = 0;
      LY::mj(t, i, m, j);
      const bool ok = LY::valid(t, i);
#pragma unroll
      for (int r = 0; r < SchedInfo<SYFX>::last; ++r) {
        const int k = LY::in_pos(j, r);
        const int ky = HY ? (2 * k < NI ? k : k + N - NI) : k;  // full-length row
        f[i * SchedInfo<SYFX>::last + r] = vt[ok ? ky * N + (QB ? GYF::band_col(m) : m) : 0];
      }
    }
  };
  cpx<T> v[FX::VALS];
  T vf[LY::VALS];
  int L = lg;
  load_rows(plane_base(L), v, tid);
  while (true) {
    // persistent form: the thread index is made opaque once per plane, so the
    // compiler recomputes the (cheap) LDS and HBM offsets instead of keeping
    // every one of them live across the loop
    int t = tid;
    if constexpr (PP) asm volatile("" : "+v"(t));
    cpx<T>* __restrict__ base = plane_base(L);
    load_v(L, vf, t);
    const int next = PP ? L + (int)gridDim.x : total;
    {
      cpx<T> o[LXF::VALS];
      EXF::reg2reg(v, plane, twxf, t, o);
      // the row registers are free: the next plane's rows go out now
      if (PP && next < total) load_rows(plane_base(next), v, t);
      if constexpr (QB == 0) {
        EXF::store_last(o, plane, t);
      } else {
        // columns beyond the band hold rounding noise only: store zeros
#pragma unroll
        for (int i = 0; i < LXF::PER; ++i) {
          if (!LXF::valid(t, i)) continue;
          int m, j;
          LXF::mj(t, i, m, j);
#pragma unroll
          for (int r = 0; r < SchedInfo<SXFX>::last; ++r) {
            if constexpr (XD) {
              // half-length frequency k: column k below N / 4, k + N / 2 above
              // (negative); k = N / 4 (|kx| = N / 4, beyond the band, rounding
              // noise only) clears the band's edge columns N / 4 and 3 N / 4;
              // columns outside the band are never read (see the inverse x)
              const int k = LXF::out_pos(j, r);
              if (2 * k == NXI) {
                plane[GX::idx(m, QB)] = cpx<T>{T(0), T(0)};
                plane[GX::idx(m, N - QB)] = cpx<T>{T(0), T(0)};
              } else {
                plane[GX::idx(m, 2 * k < NXI ? k : k + N - NXI)] = o[i * SchedInfo<SXFX>::last + r];
              }
            } else {
              const int x = LXF::out_pos(j, r);
              const bool in = x <= QB || x >= N - QB;
              plane[GX::idx(m, x)] = in ? o[i * SchedInfo<SXF>::last + r] : cpx<T>{T(0), T(0)};
              // half-height: the lower rows' columns beyond the band are zero too
              if (HY && !in) plane[GX::idx(m + NI, x)] = cpx<T>{T(0), T(0)};
            }
          }
        }
      }
    }
    __syncthreads();
    // y forward, multiply by v(G)/N_r, y inverse (hand-over in registers)
    cpx<T> oy[LY::VALS];
    EYF::lds2reg(plane, twyf, t, oy);  // ends with a barrier after its last LDS read
    if constexpr (!HY) {
#pragma unroll
      for (int i = 0; i < LY::PER; ++i) {
        if (!LY::valid(t, i)) continue;
#pragma unroll
        for (int r = 0; r < SchedInfo<SYF>::last; ++r)
          oy[i * SchedInfo<SYF>::last + r] =
              cscale(oy[i * SchedInfo<SYF>::last + r], vf[i * SchedInfo<SYF>::last + r]);
      }
      cpx<T> o[LYI::VALS];
      EYI::reg2reg(oy, plane, twyi, t, o);
      EYI::store_last(o, plane, t);
    } else {
      // the multiplied half-length spectrum goes to its full-length rows;
      // frequencies beyond the y band hold rounding noise only: zeros
#pragma unroll
      for (int i = 0; i < LY::PER; ++i) {
        if (!LY::valid(t, i)) continue;
        int m, j;
        LY::mj(t, i, m, j);
#pragma unroll
        for (int r = 0; r < SchedInfo<SYFX>::last; ++r) {
          const int k = LY::in_pos(j, r);
          const bool lo = 2 * k < NI;
          const int row = lo ? k : k + N - NI;
          const bool in = (lo ? k : NI - k) <= a.ky_max;
          plane[row * P + GYF::band_col(m)] =
              in ? cscale(oy[i * SchedInfo<SYFX>::last + r], vf[i * SchedInfo<SYFX>::last + r])
                 : cpx<T>{T(0), T(0)};
        }
      }
      // rows NI/2 .. N - NI/2 - 1 of the band columns: no half-length frequency
      for (int e = t; e < (N - NI) * MB; e += NT) {
        const int row = NI / 2 + e / MB, m = e - (e / MB) * MB;
        plane[row * P + GYF::band_col(m)] = cpx<T>{T(0), T(0)};
      }
      __syncthreads();
      cpx<T> o[LYI::VALS];
      EYI::lds2reg(plane, twyi, t, o);
      EYI::store_last(o, plane, t);
    }
    __syncthreads();
    // x inverse, results straight to HBM
    cpx<T> ox[LXI::VALS];
    if constexpr (XD) {
      // the band's columns from LDS, zeros elsewhere (never written)
      cpx<T> xi[FXI::VALS];
#pragma unroll
      for (int i = 0; i < FXI::PER; ++i) {
        if (!FXI::valid(t, i)) continue;
        int m, j;
        FXI::mj(t, i, m, j);
#pragma unroll
        for (int r = 0; r < SchedInfo<SXI>::first; ++r) {
          const int x = FXI::in_pos(j, r);
          xi[i * SchedInfo<SXI>::first + r] =
              (x <= QB || x >= N - QB) ? plane[GX::idx(m, x)] : cpx<T>{T(0), T(0)};
        }
      }
      __syncthreads();
      EXI::reg2reg(xi, plane, twxi, t, ox);
    } else {
      EXI::lds2reg(plane, twxi, t, ox);
    }
#pragma unroll
    for (int i = 0; i < LXI::PER; ++i) {
      if (!LXI::valid(t, i)) continue;
      int m, j;
      LXI::mj(t, i, m, j);
#pragma unroll
      for (int r = 0; r < SchedInfo<SXI>::last; ++r)
        base[m * N + LXI::in_pos(j, r)] = ox[i * SchedInfo<SXI>::last + r];
    }
    if (next >= total) break;
    L = next;
    __syncthreads();  // this plane's LDS reads end before the next plane's writes
  }
}

// ---------------------------------------------------------------------------
// Pass 2 for planes whose LDS copy would fill a compute unit (128^2 float32:
// 132 KB of the 160 KB): the plane is held in registers between the
// transforms and passes through a half-plane LDS buffer, so two workgroups
// share a compute unit and overlap each other's loads, barriers and stores.
//   x forward : two halves of N/2 rows, each transformed through the buffer
//               [N/2][N + 1]; results stay in registers (the last stage's
//               legs: leg r of butterfly j is column j + r N / R_last)
//   y pass    : two halves of N/2 columns: the registers of the half are
//               scattered to the buffer [N][N/2 + 1], forward y, multiply by
//               v(G)/N_r, inverse y, gathered back into the same registers
//   x inverse : two halves of rows, scattered at the x forward's positions,
//               transformed from LDS and stored to HBM.
template <typename T, int N, int NT, class SXF, class SXI, class SYF, class SYI, int NZ = N>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((2 * NT / 64 + 3) / 4)))
k_plane_h2(PassGroup grp) {
  int sys_ = 0;
  const int lg = grp.locate(xcd_remap(blockIdx.x, gridDim.x), sys_);
  const PassArgs& a = grp.a[sys_];
  constexpr int H = N / 2;
  constexpr int PX = N + 1;  // row-half buffer [H][N + 1]
  constexpr int PY = H + 1;  // column-half buffer [N][H + 1]
  using GX = Geom<T, N, H, NT, false, 1, PX>;  // sequences m = rows of the half, n = x
  using GY = Geom<T, N, H, NT, true, PY, 1>;   // sequences m = columns of the half, n = y
  using EXF = FFT<GX, false, SXF>;
  using EXI = FFT<GX, true, SXI>;
  using EYF = FFT<GY, false, SYF>;
  using EYI = FFT<GY, true, SYI>;
  using FX = FirstStage<GX, SXF>;
  using LXF = LastStage<GX, SXF>;
  using LY = LastStage<GY, SYF>;
  using LYI = LastStage<GY, SYI>;
  using LXI = LastStage<GX, SXI>;
  constexpr int RL = SchedInfo<SXF>::last;
  static_assert(N % 2 == 0 && RL % 2 == 0, "halves of rows and columns");
  static_assert(LXF::NBF == N / RL && LXF::NBF == SchedInfo<SXF>::last_span,
                "last x stage: leg r of butterfly j is column j + r N / R");
  static_assert(SchedInfo<SYI>::first == SchedInfo<SYF>::last, "fused y schedules");
  static_assert(LYI::VALS > 0 && LY::VALS == FirstStage<GY, SYI>::VALS, "fused y register maps");
  constexpr long long NR = (long long)NZ * N * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int total = a.n_active * kz_planes(NZ, a.kz_max);
  if (lg >= total) return;
  __shared__ TwEntry<T> twxf[tw_slots<T, SXF>()], twyf[tw_slots<T, SYF>()],
      twyi[tw_slots<T, SYI>()], twxi[tw_slots<T, SXI>()];
  stage_twiddles<T, SXF, NT>(twxf, a.tw_xf, tid);  // visible after the first barrier
  stage_twiddles<T, SYF, NT>(twyf, a.tw_yf, tid);
  stage_twiddles<T, SYI, NT>(twyi, a.tw_yi, tid);
  stage_twiddles<T, SXI, NT>(twxi, a.tw_xi, tid);
  const int c_ = lg / a.n_active, ai = lg - c_ * a.n_active;
  const int kz = kz_of_plane(c_, NZ, a.kz_max);
  cpx<T>* __restrict__ base = static_cast<cpx<T>*>(a.grids) + (long long)a.active[ai] * NR +
                              (long long)kz * N * N;
  const T* __restrict__ vt = static_cast<const T*>(a.vtab) + (long long)kz * N * N;

  // the x-transformed plane: row half h, the last stage's legs
  cpx<T> xr[2][LXF::VALS];
  static_for<0, 2>([&](auto hc) {
    constexpr int h = decltype(hc)::value;
    cpx<T> v[FX::VALS];
#pragma unroll
    for (int i = 0; i < FX::PER; ++i) {
      if (!FX::valid(tid, i)) continue;
      int m, j;
      FX::mj(tid, i, m, j);
#pragma unroll
      for (int r = 0; r < SchedInfo<SXF>::first; ++r)
        v[i * SchedInfo<SXF>::first + r] = base[(h * H + m) * N + FX::in_pos(j, r)];
    }
    EXF::reg2reg(v, buf, twxf, tid, xr[h]);  // the buffer is free again on return
  });
  // y pass over two column halves
  static_for<0, 2>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    static_for<0, 2>([&](auto hc) {
      constexpr int h = decltype(hc)::value;
#pragma unroll
      for (int i = 0; i < LXF::PER; ++i) {
        if (!LXF::valid(tid, i)) continue;
        int m, j;
        LXF::mj(tid, i, m, j);
#pragma unroll
        for (int r = c * RL / 2; r < (c + 1) * RL / 2; ++r)
          buf[(h * H + m) * PY + LXF::out_pos(j, r) - c * H] = xr[h][i * RL + r];
      }
    });
    __syncthreads();
    cpx<T> oy[LY::VALS];
    EYF::lds2reg(buf, twyf, tid, oy);
#pragma unroll
    for (int i = 0; i < LY::PER; ++i) {
      if (!LY::valid(tid, i)) continue;
      int m, j;
      LY::mj(tid, i, m, j);
#pragma unroll
      for (int r = 0; r < SchedInfo<SYF>::last; ++r)
        oy[i * SchedInfo<SYF>::last + r] =
            cscale(oy[i * SchedInfo<SYF>::last + r], vt[LY::in_pos(j, r) * N + c * H + m]);
    }
    {
      cpx<T> o[LYI::VALS];
      EYI::reg2reg(oy, buf, twyi, tid, o);
      EYI::store_last(o, buf, tid);
    }
    __syncthreads();
    static_for<0, 2>([&](auto hc) {
      constexpr int h = decltype(hc)::value;
#pragma unroll
      for (int i = 0; i < LXF::PER; ++i) {
        if (!LXF::valid(tid, i)) continue;
        int m, j;
        LXF::mj(tid, i, m, j);
#pragma unroll
        for (int r = c * RL / 2; r < (c + 1) * RL / 2; ++r)
          xr[h][i * RL + r] = buf[(h * H + m) * PY + LXF::out_pos(j, r) - c * H];
      }
    });
    __syncthreads();  // the buffer is rewritten next
  });
  // x inverse over two row halves, results straight to HBM
  static_for<0, 2>([&](auto hc) {
    constexpr int h = decltype(hc)::value;
    EXF::store_last(xr[h], buf, tid);
    __syncthreads();
    cpx<T> ox[LXI::VALS];
    EXI::lds2reg(buf, twxi, tid, ox);  // ends with a barrier after its last LDS read
#pragma unroll
    for (int i = 0; i < LXI::PER; ++i) {
      if (!LXI::valid(tid, i)) continue;
      int m, j;
      LXI::mj(tid, i, m, j);
#pragma unroll
      for (int r = 0; r < SchedInfo<SXI>::last; ++r)
        base[(h * H + m) * N + LXI::in_pos(j, r)] = ox[i * SchedInfo<SXI>::last + r];
    }
  });
}

// ---------------------------------------------------------------------------
// Split plane pass for grids whose plane does not fit in LDS:
// (a) FFT along x of RW consecutive rows, (b) y columns with the multiply.
template <typename T, int N, int RW, int NT, class SX, bool INV>
__global__ void __launch_bounds__(NT) k_rows(PassGroup grp) {
  int sys_ = 0;
  const int lg_ = grp.locate(xcd_remap(blockIdx.x, gridDim.x), sys_);
  const PassArgs& a = grp.a[sys_];
  constexpr int P = N + 1;
  using G = Geom<T, N, RW, NT, false, 1, P>;
  using E = FFT<G, INV, SX>;
  using F = FirstStage<G, SX>;
  using L = LastStage<G, SX>;
  constexpr long long NR = (long long)N * N * N;
  // rows (z, y) of the kept kz planes, numbered compactly; row blocks per grid
  const int nrows = kz_planes(N, a.kz_max) * N;
  const int RB = (nrows + RW - 1) / RW;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int lg = lg_;
  const int ai = lg / RB, rb = lg - ai * RB;
  const int slot = a.active[ai];
  cpx<T>* __restrict__ base = static_cast<cpx<T>*>(a.grids) + (long long)slot * NR;
  const long long row0 = (long long)rb * RW;
  // grid row of compact row c (c < nrows)
  auto grid_row = [&](long long c) {
    const int zc = (int)(c / N);
    return (long long)kz_of_plane(zc, N, a.kz_max) * N + (c - (long long)zc * N);
  };
  __shared__ TwEntry<T> twl[tw_slots<T, SX>()];
  stage_twiddles<T, SX, NT>(twl, INV ? a.tw_xi : a.tw_xf, tid);  // visible after the first barrier
  const TwEntry<T>* tw = twl;
  cpx<T> v[F::VALS];
#pragma unroll
  for (int i = 0; i < F::PER; ++i) {
    if (!F::valid(tid, i)) continue;
    int m, j;
    F::mj(tid, i, m, j);
    const bool rv = row0 + m < nrows;
    const long long gr = rv ? grid_row(row0 + m) : 0;
#pragma unroll
    for (int r = 0; r < SchedInfo<SX>::first; ++r)
      v[i * SchedInfo<SX>::first + r] =
          rv ? base[gr * N + F::in_pos(j, r)] : cpx<T>{T(0), T(0)};
  }
  cpx<T> o[L::VALS];
  E::reg2reg(v, lds, tw, tid, o);
#pragma unroll
  for (int i = 0; i < L::PER; ++i) {
    if (!L::valid(tid, i)) continue;
    int m, j;
    L::mj(tid, i, m, j);
    if (row0 + m >= nrows) continue;
    const long long gr = grid_row(row0 + m);
#pragma unroll
    for (int r = 0; r < SchedInfo<SX>::last; ++r)
      base[gr * N + L::in_pos(j, r)] = o[i * SchedInfo<SX>::last + r];
  }
}

template <typename T, int N, int W, int NT, class SYF, class SYI>
__global__ void __launch_bounds__(NT) k_cols_conv(PassGroup grp) {
  int sys_ = 0;
  const int lg_ = grp.locate(xcd_remap(blockIdx.x, gridDim.x), sys_);
  const PassArgs& a = grp.a[sys_];
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
  __shared__ TwEntry<T> twf[tw_slots<T, SYF>()], twi[tw_slots<T, SYI>()];
  const int tid = threadIdx.x;
  stage_twiddles<T, SYF, NT>(twf, a.tw_yf, tid);  // visible after the first barrier
  stage_twiddles<T, SYI, NT>(twi, a.tw_yi, tid);
  const int lg = lg_;
  const int per_grid = kz_planes(N, a.kz_max) * NXB;  // kept planes x column blocks
  const int ai = lg / per_grid, rem = lg - ai * per_grid;
  const int zc = rem / NXB, x0 = (rem - zc * NXB) * W;
  const int z = kz_of_plane(zc, N, a.kz_max);
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
  EF::reg2reg(v, lds, twf, tid, o);
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
  EI::reg2reg(o, lds, twi, tid, b);
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

// Threads of the pair_fwd (FWD) and inv_acc passes.  float32: 256 for the
// product pass (fewer, longer wavefronts measured fastest), and for the
// accumulation pass 512, or 1024 for bricks of more than 1536 points (3
// points per thread keep the tile's psi and accumulators within 128
// registers, so that whole workgroups fill the compute unit).  float64: 2
// brick points per thread, or 4 for bricks too large for 768 threads (more
// threads per workgroup would cap the registers at 128 and spill).
template <typename T, int N, int W, bool FWD>
constexpr int pencil_threads() {
  if constexpr (sizeof(T) == 4) {
    return FWD ? 256 : (N * W > 1536 ? 1024 : 512);
  } else {
    return N * W / 2 > 768 ? (N * W + 3) / 4 : (N * W + 1) / 2;
  }
}
// psi_J block in LDS and next-step prefetch in inv_acc: float32 bricks of up
// to 1728 points (measured faster there; larger bricks spill with it).
template <typename T, int N, int W>
constexpr bool pencil_prefetch() {
  return sizeof(T) == 4 && N * W <= 1728;
}
template <int... R>
constexpr void fill_radices(int* dst, int& n, Sched<R...>) {
  const int r[] = {R...};
  n = (int)sizeof...(R);
  for (int i = 0; i < n; ++i) dst[i] = r[i];
}

// Fused three-pass pipeline: W-wide z bricks, TT-orbital tiles, plane
// kernel of NTQ threads with the plane in LDS.
template <typename T, int N, int W, int TT, class SZF, class SZI, int NTQ, class SXF, class SXI,
          class SYF, class SYI, bool SW = false,
          int NTF = pencil_threads<T, N, W, true>(), int NTI = pencil_threads<T, N, W, false>(),
          bool PJL = pencil_prefetch<T, N, W>(), bool PF = pencil_prefetch<T, N, W>(),
          bool PIL = false, bool PP = false, int NZ = N, int FLI = 0,
          class SZH = typename HalfZ<NZ / 2>::type, int PM = 1, bool GMP = false>
struct FusedPipeline {
  // PM: plane kernel (1: the plane in LDS, k_plane_conv; 2: the plane in
  // registers with a half-plane LDS buffer, two workgroups per compute unit,
  // k_plane_h2)
  static_assert(PM == 1 || (PM == 2 && !PP && !SW && NZ == N), "plane kernel mode");
  // FLI: inv_acc flat loads (0: none; 1: two grids per transform; 4: the four
  // grids of a tile row per transform)
  static_assert(FLI == 0 || FLI == 1 || FLI == 4, "flat-load mode");
  static_assert(FLI == 0 || PF, "flat loads are a form of the prefetching accumulation");
  static constexpr bool FLB = FLI != 0;
  static constexpr int NGI = FLI == 4 ? 4 : 2;
  static constexpr size_t lds =
      PM == 2 ? (size_t)((N / 2) * (N + 1) > N * (N / 2 + 1) ? (N / 2) * (N + 1) : N * (N / 2 + 1)) *
                    sizeof(cpx<T>)
              : (size_t)N * (N + 1) * sizeof(cpx<T>);
  // band of the plane kernel's column-pruned instantiation (float32 cubic
  // grids from 64 up to 120, plain layouts): |kx| <= N / 4, the band of
  // orbitals at half the grid's plane-wave reach (a twofold oversampled grid)
  static constexpr int QB = (sizeof(T) == 4 && NZ == N && N >= 64 && N <= 120 && !SW)
                                ? N / 4 : 0;
  // persistent plane kernel: one workgroup per plane slot of the device
  static int plane_grid(int planes) {
    if (!PP) return planes;
    static const int slots = [] {
      int d = 0, cu = 0;
      if (hipGetDevice(&d) != hipSuccess ||
          hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess ||
          cu <= 0)
        cu = 256;
      const int per_cu = (int)((160 * 1024) / (lds + 4096));
      return cu * (per_cu > 0 ? per_cu : 1);
    }();
    return planes < slots ? planes : slots;
  }
  // half-length forward z for band-limited plans (float32)
  static constexpr bool HZOK = sizeof(T) == 4 && NZ % 2 == 0 && !std::is_void_v<SZH>;
  // half-height plane input (band columns, cubic grids; the half-length y
  // transforms take the half-length z schedule and its twiddles)
  static constexpr bool HYOK = QB > 0 && HZOK && NZ == N && N % 4 == 0 && PM == 1;
  // the same test as the host's (run_exchange): every system of the group has
  // its x band within the band columns and its y band within N / 4
  static bool use_hy(const PassGroup& g) {
    if constexpr (!HYOK) {
      return false;
    } else {
      bool hy = true;
      for (int i = 0; i < g.count; ++i)
        hy = hy && g.a[i].kx_max <= QB && g.a[i].ky_max <= (N / 2 - 1) / 2;
      return hy;
    }
  }
  // half-width plane input as well (the host's half_x): every x band within
  // N / 4 - 1, so that the even x points sample it exactly
  static bool use_xd(const PassGroup& g) {
    if constexpr (!HYOK) {
      return false;
    } else {
      bool xd = use_hy(g);
      for (int i = 0; i < g.count; ++i) xd = xd && g.a[i].kx_max <= (N / 2 - 1) / 2;
      return xd;
    }
  }
  template <bool HZ, bool HY, bool XD>
  static void fwd_launch(const PassGroup& g, int nb, hipStream_t s) {
    if (g.a[0].perm)
      hipLaunchKernelGGL((k_pair_fwd<T, N, W, NTF, TT, SZF, PIL, true, NZ, HZ, SZH, HY, XD>),
                         dim3(nb), dim3(NTF), 0, s, g);
    else
      hipLaunchKernelGGL((k_pair_fwd<T, N, W, NTF, TT, SZF, PIL, false, NZ, HZ, SZH, HY, XD>),
                         dim3(nb), dim3(NTF), 0, s, g);
  }
  template <bool HZ>
  static void fwd_rows(const PassGroup& g, int nb, hipStream_t s) {
    if constexpr (HYOK) {
      if (use_xd(g))
        fwd_launch<HZ, true, true>(g, nb, s);
      else if (use_hy(g))
        fwd_launch<HZ, true, false>(g, nb, s);
      else
        fwd_launch<HZ, false, false>(g, nb, s);
    } else {
      fwd_launch<HZ, false, false>(g, nb, s);
    }
  }
  static void pair_fwd(const PassGroup& g, int nb, hipStream_t s) {
    if constexpr (HZOK) {
      bool half = true;
      for (int i = 0; i < g.count; ++i) half = half && g.a[i].kz_max <= (NZ / 2 - 1) / 2;
      if (half) {
        fwd_rows<true>(g, nb, s);
        return;
      }
    }
    fwd_rows<false>(g, nb, s);
  }
  static void plane(const PassGroup& g, int nb, hipStream_t s) {
    if constexpr (PM == 2) {
      hipLaunchKernelGGL((k_plane_h2<T, N, NTQ, SXF, SXI, SYF, SYI, NZ>), dim3(nb), dim3(NTQ), lds,
                         s, g);
      return;
    }
    if constexpr (QB > 0) {
      bool band = true;
      for (int i = 0; i < g.count; ++i) band = band && g.a[i].kx_max <= QB;
      if (band) {
        if constexpr (HYOK) {
          if (use_xd(g)) {
            hipLaunchKernelGGL(
                (k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, QB, GMP, true, SZH, true>),
                dim3(plane_grid(nb)), dim3(NTQ), lds, s, g);
            return;
          }
          if (use_hy(g)) {
            hipLaunchKernelGGL(
                (k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, QB, GMP, true, SZH>),
                dim3(plane_grid(nb)), dim3(NTQ), lds, s, g);
            return;
          }
        }
        hipLaunchKernelGGL((k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, QB, GMP>),
                           dim3(plane_grid(nb)), dim3(NTQ), lds, s, g);
        return;
      }
    }
    hipLaunchKernelGGL((k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, 0, GMP>),
                       dim3(plane_grid(nb)), dim3(NTQ), lds, s, g);
  }
  // screened (perm) and band-limited (kz_max < NZ / 2) plans take their own
  // instantiations
  template <bool ACC, bool SCR>
  static void inv_launch(const PassGroup& g, int nb, hipStream_t s) {
    // band-limited plans: float32 takes zero-block loads while at least 3/4
    // of the planes are kept and skipped loads below that; float64 (one
    // workgroup per compute unit, registers tight) always skips (measured at
    // 93 of 96 planes and at 29..57 of 64..120)
    const int kept = kz_planes(NZ, g.a[0].kz_max);
    if (kept == NZ) {
      hipLaunchKernelGGL((k_inv_acc<T, N, W, NTI, TT, SZI, ACC, PJL, PF, SCR, NZ, 0, FLB, NGI>), dim3(nb),
                         dim3(NTI), 0, s, g);
      return;
    }
    if constexpr (sizeof(T) == 4) {
      if (4 * kept >= 3 * NZ) {
        hipLaunchKernelGGL((k_inv_acc<T, N, W, NTI, TT, SZI, ACC, PJL, PF, SCR, NZ, 1, FLB, NGI>), dim3(nb),
                           dim3(NTI), 0, s, g);
        return;
      }
    }
    hipLaunchKernelGGL((k_inv_acc<T, N, W, NTI, TT, SZI, ACC, PJL, PF, SCR, NZ, 2, FLB, NGI>), dim3(nb),
                       dim3(NTI), 0, s, g);
  }
  template <bool ACC>
  static void inv_pass(const PassGroup& g, int nb, hipStream_t s) {
    if (g.a[0].perm)
      inv_launch<ACC, true>(g, nb, s);
    else
      inv_launch<ACC, false>(g, nb, s);
  }
  static void inv_acc(const PassGroup& g, int nb, hipStream_t s) { inv_pass<true>(g, nb, s); }
  static void inv_energy(const PassGroup& g, int nb, hipStream_t s) { inv_pass<false>(g, nb, s); }
  static hipError_t prepare() {
    if constexpr (PM == 2)
      return hipFuncSetAttribute(
          reinterpret_cast<const void*>(&k_plane_h2<T, N, NTQ, SXF, SXI, SYF, SYI, NZ>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, 0, GMP>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess || QB == 0) return e;
    e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, QB, GMP>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if constexpr (HYOK) {
      if (e == hipSuccess)
        e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(
                &k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, QB, GMP, true, SZH>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e == hipSuccess)
        e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(
                &k_plane_conv<T, N, NTQ, SXF, SXI, SYF, SYI, SW, PP, NZ, QB, GMP, true, SZH, true>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    return e;
  }
  static Variant describe(const char* name) {
    Variant v{};
    v.name = name;
    v.n = N;
    v.nz = NZ;
    v.prec = sizeof(T) == 8 ? 1 : 0;
    v.brick = W;
    v.tile = TT;
    v.max_rows = PIL ? TT : kMaxRows;
    v.nt_fwd = NTF;
    v.nt_acc = NTI;
    v.nt_plane = NTQ;
    v.nt_cols = 0;
    v.plane_mode = 0;
    v.rows_per_wg = 0;
    v.persistent = PP;
    fill_radices(v.zf, v.nzf, SZF{});
    fill_radices(v.zi, v.nzi, SZI{});
    fill_radices(v.xf, v.nxf, SXF{});
    fill_radices(v.xi, v.nxi, SXI{});
    fill_radices(v.yf, v.nyf, SYF{});
    fill_radices(v.yi, v.nyi, SYI{});
    v.nzh = 0;
    if constexpr (HZOK) fill_radices(v.zh, v.nzh, SZH{});
    v.qb = QB;
    v.hy = HYOK;
    v.xd = HYOK;
    v.plane_lds = lds;
    v.pair_fwd = &pair_fwd;
    v.plane = &plane;
    v.inv_acc = &inv_acc;
    v.inv_energy = &inv_energy;
    v.prepare = &prepare;
    return v;
  }
};

// Split pipeline (plane too large for LDS): RW-row x kernels of NTQ threads,
// y-column kernel of NTC threads.
template <typename T, int N, int W, int NTC, int TT, class SZF, class SZI, int RW, int NTQ,
          class SXF, class SXI, class SYF, class SYI,
          int NTF = pencil_threads<T, N, W, true>(), int NTI = pencil_threads<T, N, W, false>(),
          bool PJL = false, bool PF = false, bool PIL = false>
struct SplitPipeline {
  static constexpr size_t lds = (size_t)RW * (N + 1) * sizeof(cpx<T>);
  static void pair_fwd(const PassGroup& g, int nb, hipStream_t s) {
    if (g.a[0].perm)
      hipLaunchKernelGGL((k_pair_fwd<T, N, W, NTF, TT, SZF, PIL, true>), dim3(nb), dim3(NTF), 0, s, g);
    else
      hipLaunchKernelGGL((k_pair_fwd<T, N, W, NTF, TT, SZF, PIL, false>), dim3(nb), dim3(NTF), 0, s, g);
  }
  static void rows_fwd(const PassGroup& g, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_rows<T, N, RW, NTQ, SXF, false>), dim3(nb), dim3(NTQ), lds, s, g);
  }
  static void rows_inv(const PassGroup& g, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_rows<T, N, RW, NTQ, SXI, true>), dim3(nb), dim3(NTQ), lds, s, g);
  }
  static void cols_conv(const PassGroup& g, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_cols_conv<T, N, W, NTC, SYF, SYI>), dim3(nb), dim3(NTC), 0, s, g);
  }
  // screened (perm) and band-limited (kz_max < N / 2: pruned loads skipped)
  // plans take their own instantiations
  template <bool ACC, bool SCR>
  static void inv_launch(const PassGroup& g, int nb, hipStream_t s) {
    if (kz_planes(N, g.a[0].kz_max) == N)
      hipLaunchKernelGGL((k_inv_acc<T, N, W, NTI, TT, SZI, ACC, PJL, PF, SCR, N, 0>), dim3(nb),
                         dim3(NTI), 0, s, g);
    else
      hipLaunchKernelGGL((k_inv_acc<T, N, W, NTI, TT, SZI, ACC, PJL, PF, SCR, N, 2>), dim3(nb),
                         dim3(NTI), 0, s, g);
  }
  static void inv_acc(const PassGroup& g, int nb, hipStream_t s) {
    if (g.a[0].perm)
      inv_launch<true, true>(g, nb, s);
    else
      inv_launch<true, false>(g, nb, s);
  }
  static void inv_energy(const PassGroup& g, int nb, hipStream_t s) {
    if (g.a[0].perm)
      inv_launch<false, true>(g, nb, s);
    else
      inv_launch<false, false>(g, nb, s);
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
    v.nz = N;
    v.prec = sizeof(T) == 8 ? 1 : 0;
    v.brick = W;
    v.tile = TT;
    v.max_rows = PIL ? TT : kMaxRows;
    v.nt_fwd = NTF;
    v.nt_acc = NTI;
    v.nt_plane = NTQ;
    v.nt_cols = NTC;
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
