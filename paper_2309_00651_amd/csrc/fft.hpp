// Mixed-radix Stockham FFT engine for CDNA4 workgroups.
//
// A workgroup of NT threads transforms M independent complex sequences of
// length N at once.  Each stage of radix R runs M*N/R butterflies: a thread
// gathers the R legs of its butterflies into registers, applies the stage
// twiddles, runs an unrolled radix-R codelet and scatters the results.
// Between stages the data pass through LDS (all threads read, barrier,
// compute, write, barrier); the first stage may take its inputs straight
// from registers (loaded from HBM by the caller) and the last stage leaves its
// outputs in registers, so a kernel can fuse a pointwise producer before the
// transform and a consumer after it.
//
// Stage s (radix R, span Ns = product of the earlier radices), butterfly j:
//   inputs  x[j + r N/R]                                   r = 0..R-1
//   twiddle W_{Ns R}^{r (j mod Ns)}   (W_n = exp(-2 pi i / n), conjugated
//                                      for the inverse transform)
//   outputs y[(j div Ns) Ns R + (j mod Ns) + r Ns]
// After the last stage the outputs are in natural order, and butterfly j of
// the last stage holds X[j + r N/R_last].
//
// Butterflies are numbered q = tid + i*NT (i < PER) and mapped to
// (sequence m, butterfly j) either m-fastest (MFAST: neighbouring threads own
// neighbouring sequences, used for pencils whose sequences are adjacent in
// memory) or j-fastest (neighbouring threads walk along one sequence, used
// for contiguous rows).  LDS element (m, n) lives at m*TS + n*ES.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "trig.hpp"

#define HFX_HD __host__ __device__ __forceinline__

namespace hfx {

template <typename T>
struct cpx {
  T re, im;
};

template <typename T>
HFX_HD cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
HFX_HD cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
HFX_HD cpx<T> cscale(cpx<T> a, T s) {
  return {a.re * s, a.im * s};
}
// a * (-i)
template <typename T>
HFX_HD cpx<T> mul_mi(cpx<T> a) {
  return {a.im, -a.re};
}
// a * (+i)
template <typename T>
HFX_HD cpx<T> mul_pi(cpx<T> a) {
  return {-a.im, a.re};
}
// a * w, or a * conj(w) when CONJ
template <bool CONJ, typename T>
HFX_HD cpx<T> cmul(cpx<T> a, cpx<T> w) {
  if constexpr (CONJ) {
    return {a.re * w.re + a.im * w.im, a.im * w.re - a.re * w.im};
  } else {
    return {a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
  }
}

// x * c for a compile-time constant c.  In float32 the constant is carried as
// hi + lo (hi = fl32(c), lo = fl32(c - hi)) and the product is formed as
// fma(x, hi, x * lo): plain rounding of constants such as sqrt(1/2) or
// sin(2 pi / 3) is one-sided and would bias the gain of every transform by
// ~1e-8 per codelet, which accumulates over the six passes of a convolution.
template <typename T>
HFX_HD T mulk(T x, double c) {
  if constexpr (sizeof(T) == 8) {
    return x * c;
  } else {
    const float hi = (float)c;
    const float lo = (float)(c - (double)hi);
    return __builtin_fmaf(x, hi, x * lo);
  }
}

// Low part of a float32 constant split hi + lo.  A remainder below 2^-46 |c|
// is the float64 evaluation's own error of a constant that float32 holds
// exactly (0.5 = sin(pi/6) comes out one float64 ulp low): taken as zero, so
// the product needs no correction term.
HFX_HD float lo_part(double c, float hi) {
  const double lo = c - (double)hi;
  const double ac = c < 0 ? -c : c;
  return (lo < 0 ? -lo : lo) <= ac * 0x1p-46 ? 0.0f : (float)lo;
}

// A float32 power of two: its products are exact, with no bits below the
// last place.
HFX_HD bool pow2f(float h) { return (__builtin_bit_cast(unsigned, h) & 0x7fffffu) == 0u; }

// x c + y d (+ z) for compile-time constants c, d.  In float32 both
// constants are split hi + lo as in mulk, and the sum is one chain of fused
// multiply-adds: the low terms enter the fma of a product x c_hi or y d_hi
// that is not exact (c_hi not a power of two), whose bits below the last
// place make its rounding unbiased.  Added to an exact value (z, or a
// product by 0.5) they would fall below half a unit in the last place and be
// dropped, always in the same direction: the one-sided error the split is
// there to remove.  3-4 instructions where two mulk products and their sum
// take 5; two roundings of significant size instead of three.  z is added
// last.
template <typename T>
HFX_HD T dotk(T x, double c, T y, double d) {
  if constexpr (sizeof(T) == 8) {
    return x * c + y * d;
  } else {
    float ch = (float)c, dh = (float)d;
    if (pow2f(dh) && !pow2f(ch)) {
      const T tx = x;
      x = y;
      y = tx;
      const double tc = c;
      c = d;
      d = tc;
      const float th = ch;
      ch = dh;
      dh = th;
    }
    const float cl = lo_part(c, ch), dl = lo_part(d, dh);
    if (dl != 0.0f) {
      const float s = cl != 0.0f ? __builtin_fmaf(x, cl, y * dl) : y * dl;
      return __builtin_fmaf(x, ch, __builtin_fmaf(y, dh, s));
    }
    if (cl != 0.0f) return __builtin_fmaf(y, dh, __builtin_fmaf(x, ch, x * cl));
    return __builtin_fmaf(x, ch, y * dh);
  }
}
template <typename T>
HFX_HD T dotk(T x, double c, T y, double d, T z) {
  if constexpr (sizeof(T) == 8) {
    return z + x * c + y * d;
  } else {
    return z + dotk(x, c, y, d);
  }
}

// Stage twiddle table entry.  float32 tables hold norm-optimised values
// (unit_f32 in twiddle.hpp), so a plain complex product keeps the transform
// gain unbiased.
template <typename T>
struct TwEntry {
  cpx<T> w;
};

template <bool CONJ, typename T>
HFX_HD cpx<T> twmul(cpx<T> a, const TwEntry<T>& t) {
  return cmul<CONJ>(a, t.w);
}

template <int B, int E, class F>
HFX_HD void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// ---------------------------------------------------------------------------
// a * W_N^K with W_N = exp(-2 pi i / N) (forward) or exp(+2 pi i / N) (INV);
// trivial and eighth-turn rotations are special-cased at compile time.
template <int N, int K, bool INV, typename T>
HFX_HD cpx<T> rot(cpx<T> a) {
  constexpr int k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (2 * k == N) {
    return {-a.re, -a.im};
  } else if constexpr (4 * k == N) {
    return INV ? mul_pi(a) : mul_mi(a);
  } else if constexpr (4 * k == 3 * N) {
    return INV ? mul_mi(a) : mul_pi(a);
  } else if constexpr ((8 * k) % N == 0) {
    // odd multiple of pi/4: both parts of W have magnitude sqrt(1/2)
    constexpr SinCos sc = sincos_2pi(k, N);
    constexpr double h = 0.70710678118654752440084436210484903928;
    constexpr int sgc = sc.c > 0 ? 1 : -1;
    constexpr int sgs = (INV ? 1 : -1) * (sc.s > 0 ? 1 : -1);  // sign of Im W
    const T x = (sgc > 0 ? a.re : -a.re) - (sgs > 0 ? a.im : -a.im);
    const T y = (sgs > 0 ? a.re : -a.re) + (sgc > 0 ? a.im : -a.im);
    return {mulk(x, h), mulk(y, h)};
  } else {
    constexpr SinCos sc = sincos_2pi(k, N);
    constexpr double c = sc.c;
    constexpr double s = INV ? sc.s : -sc.s;
    return {dotk(a.re, c, a.im, -s), dotk(a.re, s, a.im, c)};
  }
}

// ---------------------------------------------------------------------------
// Radix-R codelets: v[k] <- sum_n v[n] W_R^{nk}, in registers.
template <int R, bool INV, typename T>
struct DFT;

template <bool INV, typename T>
struct DFT<1, INV, T> {
  HFX_HD static void run(cpx<T>*) {}
};

template <bool INV, typename T>
struct DFT<2, INV, T> {
  HFX_HD static void run(cpx<T>* v) {
    const cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <bool INV, typename T>
struct DFT<3, INV, T> {
  HFX_HD static void run(cpx<T>* v) {
    constexpr double s3 = 0.86602540378443864676372317075293618;  // sin(2pi/3)
    const cpx<T> t = v[1] + v[2];
    const cpx<T> d0 = v[1] - v[2];
    const cpx<T> d = {mulk(d0.re, s3), mulk(d0.im, s3)};
    const cpx<T> m = {v[0].re - T(0.5) * t.re, v[0].im - T(0.5) * t.im};
    v[0] = v[0] + t;
    const cpx<T> id = mul_pi(d);  // i * s3 * (v1 - v2)
    if constexpr (INV) {
      v[1] = m + id;
      v[2] = m - id;
    } else {
      v[1] = m - id;
      v[2] = m + id;
    }
  }
};

template <bool INV, typename T>
struct DFT<4, INV, T> {
  HFX_HD static void run(cpx<T>* v) {
    const cpx<T> a0 = v[0] + v[2], a1 = v[0] - v[2];
    const cpx<T> b0 = v[1] + v[3], b1 = v[1] - v[3];
    const cpx<T> ib1 = mul_pi(b1);
    v[0] = a0 + b0;
    v[2] = a0 - b0;
    if constexpr (INV) {
      v[1] = a1 + ib1;
      v[3] = a1 - ib1;
    } else {
      v[1] = a1 - ib1;
      v[3] = a1 + ib1;
    }
  }
};

template <bool INV, typename T>
struct DFT<5, INV, T> {
  HFX_HD static void run(cpx<T>* v) {
    constexpr double c1 = 0.30901699437494742410229341718281906;   // cos(2pi/5)
    constexpr double c2 = -0.80901699437494742410229341718281906;  // cos(4pi/5)
    constexpr double s1 = 0.95105651629515357211643933337938214;   // sin(2pi/5)
    constexpr double s2 = 0.58778525229247312916870595463907277;   // sin(4pi/5)
    const cpx<T> a1 = v[1] + v[4], b1 = v[1] - v[4];
    const cpx<T> a2 = v[2] + v[3], b2 = v[2] - v[3];
    const cpx<T> x0 = v[0];
    const cpx<T> p1 = {dotk(a1.re, c1, a2.re, c2, x0.re), dotk(a1.im, c1, a2.im, c2, x0.im)};
    const cpx<T> p2 = {dotk(a1.re, c2, a2.re, c1, x0.re), dotk(a1.im, c2, a2.im, c1, x0.im)};
    const cpx<T> q1 = {dotk(b1.re, s1, b2.re, s2), dotk(b1.im, s1, b2.im, s2)};
    const cpx<T> q2 = {dotk(b1.re, s2, b2.re, -s1), dotk(b1.im, s2, b2.im, -s1)};
    const cpx<T> iq1 = mul_pi(q1), iq2 = mul_pi(q2);
    v[0] = x0 + a1 + a2;
    if constexpr (INV) {
      v[1] = p1 + iq1;
      v[4] = p1 - iq1;
      v[2] = p2 + iq2;
      v[3] = p2 - iq2;
    } else {
      v[1] = p1 - iq1;
      v[4] = p1 + iq1;
      v[2] = p2 - iq2;
      v[3] = p2 + iq2;
    }
  }
};

// Composite radix P*Q: inputs n = Q n1 + n2, outputs k = k1 + P k2.
//   step 1: DFT_P over n1 for each n2, times W_{PQ}^{n2 k1}
//   step 2: DFT_Q over n2 for each k1
template <int P, int Q, bool INV, typename T>
struct DFTPQ {
  HFX_HD static void run(cpx<T>* v) {
    cpx<T> t[P * Q];
    static_for<0, Q>([&](auto n2) {
      cpx<T> a[P];
      static_for<0, P>([&](auto n1) { a[n1] = v[Q * n1 + n2]; });
      DFT<P, INV, T>::run(a);
      static_for<0, P>([&](auto k1) {
        t[n2 * P + k1] = rot<P * Q, decltype(n2)::value * decltype(k1)::value, INV>(a[k1]);
      });
    });
    static_for<0, P>([&](auto k1) {
      cpx<T> b[Q];
      static_for<0, Q>([&](auto n2) { b[n2] = t[n2 * P + k1]; });
      DFT<Q, INV, T>::run(b);
      static_for<0, Q>([&](auto k2) { v[k1 + P * k2] = b[k2]; });
    });
  }
};

template <bool INV, typename T> struct DFT<6, INV, T> : DFTPQ<3, 2, INV, T> {};
template <bool INV, typename T> struct DFT<8, INV, T> : DFTPQ<2, 4, INV, T> {};
template <bool INV, typename T> struct DFT<9, INV, T> : DFTPQ<3, 3, INV, T> {};
template <bool INV, typename T> struct DFT<10, INV, T> : DFTPQ<2, 5, INV, T> {};
template <bool INV, typename T> struct DFT<12, INV, T> : DFTPQ<3, 4, INV, T> {};
template <bool INV, typename T> struct DFT<15, INV, T> : DFTPQ<3, 5, INV, T> {};
template <bool INV, typename T> struct DFT<16, INV, T> : DFTPQ<4, 4, INV, T> {};

// ---------------------------------------------------------------------------
// Geometry of one batched transform inside a workgroup.
// SWZ: LDS index swizzle for a square plane with pitch P stored [y][x]:
//   0 none: element (m, n) at m*TS + n*ES
//   1 rows (m = y, n = x) and 2 columns (m = x, n = y): element (y, x) at
//     y*P + (x ^ ((x >> 3) & 7)), an XOR inside each block of 8 along x that
//     spreads the stride-8 first-stage writes of the row transforms over the
//     banks without extra LDS (needs N % 8 == 0).
//   3 a band of columns of a plane BW points wide (BW = N unless the columns
//     are transformed at another length): M = 2Q + 1 sequences m are the
//     columns x = 0..Q and BW-Q..BW-1 (m > Q maps to x = m + BW - M); element
//     n of column m at n*ES + x (TS = 1).
template <typename T_, int N_, int M_, int NT_, bool MFAST_, int ES_, int TS_, int SWZ_ = 0,
          int BW_ = N_>
struct Geom {
  using T = T_;
  static constexpr int N = N_;     // transform length
  static constexpr int M = M_;     // number of sequences
  static constexpr int NT = NT_;   // threads in the workgroup
  static constexpr bool MFAST = MFAST_;
  static constexpr int ES = ES_;   // LDS stride between elements of a sequence
  static constexpr int TS = TS_;   // LDS stride between sequences
  static constexpr int SWZ = SWZ_;
  static constexpr int BW = BW_;
  // column of sequence m in a band geometry (SWZ == 3)
  HFX_HD static int band_col(int m) { return m <= (M - 1) / 2 ? m : m + BW - M; }
  HFX_HD static int idx(int m, int n) {
    if constexpr (SWZ == 1) {
      return m * TS + (n ^ ((n >> 3) & 7));
    } else if constexpr (SWZ == 2) {
      return n * ES + (m ^ ((m >> 3) & 7));
    } else if constexpr (SWZ == 3) {
      return n * ES + band_col(m);
    } else {
      return m * TS + n * ES;
    }
  }
};

template <class G, int R, int NS>
struct Stage {
  using T = typename G::T;
  static_assert(G::N % R == 0, "radix must divide the length");
  static constexpr int NBF = G::N / R;        // butterflies per sequence
  static constexpr int NB = G::M * NBF;       // butterflies per stage
  static constexpr int PER = (NB + G::NT - 1) / G::NT;
  static constexpr bool EXACT = (NB % G::NT) == 0;
  static constexpr int VALS = PER * R;        // complex registers per thread

  HFX_HD static bool valid(int tid, int i) {
    return EXACT || (tid + i * G::NT) < NB;
  }
  HFX_HD static void mj(int tid, int i, int& m, int& j) {
    const int q = tid + i * G::NT;
    if constexpr (G::MFAST) {
      m = q % G::M;
      j = q / G::M;
    } else {
      j = q % NBF;
      m = q / NBF;
    }
  }
  // position inside the sequence of input leg r of butterfly j
  HFX_HD static int in_pos(int j, int r) { return j + r * NBF; }
  // position of output leg r of butterfly j
  HFX_HD static int out_pos(int j, int r) {
    return (j / NS) * NS * R + (j % NS) + r * NS;
  }

  // twiddles + codelet on registers v[PER*R]; tw holds W_{NS R}^{r k}
  // at tw[k*(R-1) + r-1] (forward sign), conjugated here for INV.
  template <bool INV>
  HFX_HD static void compute(cpx<T>* v, int tid, const TwEntry<T>* __restrict__ tw) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (!valid(tid, i)) continue;
      if constexpr (NS > 1) {
        int m, j;
        mj(tid, i, m, j);
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[i * R + r] = twmul<INV>(v[i * R + r], tw[k * (R - 1) + r - 1]);
        }
      }
      DFT<R, INV, T>::run(v + i * R);
    }
  }

  HFX_HD static void read(cpx<T>* v, const cpx<T>* lds, int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (!valid(tid, i)) continue;
      int m, j;
      mj(tid, i, m, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i * R + r] = lds[G::idx(m, in_pos(j, r))];
    }
  }

  HFX_HD static void write(const cpx<T>* v, cpx<T>* lds, int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (!valid(tid, i)) continue;
      int m, j;
      mj(tid, i, m, j);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[G::idx(m, out_pos(j, r))] = v[i * R + r];
    }
  }
};

template <int... Rs>
struct Sched {};

template <class S>
struct SchedInfo;
template <int R0, int... Rs>
struct SchedInfo<Sched<R0, Rs...>> {
  static constexpr int first = R0;
  static constexpr int count = 1 + sizeof...(Rs);
  static constexpr int radices[count] = {R0, Rs...};
  static constexpr int last = radices[count - 1];
  static constexpr int product = (R0 * ... * Rs);
  // span of the last stage
  static constexpr int last_span = product / last;
  // number of twiddle entries (stages with span > 1)
  static constexpr int tw_count() {
    int n = 0, ns = 1;
    for (int s = 0; s < count; ++s) {
      if (ns > 1) n += ns * (radices[s] - 1);
      ns *= radices[s];
    }
    return n;
  }
};

template <class G, class S>
using FirstStage = Stage<G, SchedInfo<S>::first, 1>;
template <class G, class S>
using LastStage = Stage<G, SchedInfo<S>::last, SchedInfo<S>::last_span>;

// Stages 1..end: read from LDS, compute, write to LDS (or keep the final
// stage in registers `out`).  A barrier follows the final read, so the
// caller may write LDS again as soon as this returns.
template <class G, bool INV, int NS, int TWOFF, int R, int... Rest>
__device__ __forceinline__ void fft_tail(cpx<typename G::T>* lds,
                                         const TwEntry<typename G::T>* __restrict__ tw, int tid,
                                         cpx<typename G::T>* out) {
  using St = Stage<G, R, NS>;
  cpx<typename G::T> v[St::VALS];
  St::read(v, lds, tid);
  __syncthreads();
  St::template compute<INV>(v, tid, tw + TWOFF);
  if constexpr (sizeof...(Rest) > 0) {
    St::write(v, lds, tid);
    __syncthreads();
    fft_tail<G, INV, NS * R, TWOFF + NS * (R - 1), Rest...>(lds, tw, tid, out);
  } else {
#pragma unroll
    for (int e = 0; e < St::VALS; ++e) out[e] = v[e];
  }
}

template <class G, bool INV, class S>
struct FFT;

template <class G, bool INV, int R0, int... Rest>
struct FFT<G, INV, Sched<R0, Rest...>> {
  using T = typename G::T;
  using S = Sched<R0, Rest...>;
  using First = Stage<G, R0, 1>;
  using Last = LastStage<G, S>;

  // Stage-0 inputs in registers `v` (First::VALS values, element map of
  // First), outputs in registers `out` (Last::VALS, element map of Last).
  // LDS must hold M*N elements with the geometry's strides.
  __device__ __forceinline__ static void reg2reg(cpx<T>* v, cpx<T>* lds,
                                                 const TwEntry<T>* __restrict__ tw, int tid,
                                                 cpx<T>* out) {
    First::template compute<INV>(v, tid, tw);
    if constexpr (sizeof...(Rest) == 0) {
#pragma unroll
      for (int e = 0; e < First::VALS; ++e) out[e] = v[e];
    } else {
      First::write(v, lds, tid);
      __syncthreads();
      fft_tail<G, INV, R0, 0, Rest...>(lds, tw, tid, out);
    }
  }

  // Stage-0 inputs from LDS (the caller has synchronised), outputs in registers.
  __device__ __forceinline__ static void lds2reg(cpx<T>* lds, const TwEntry<T>* __restrict__ tw,
                                                 int tid, cpx<T>* out) {
    cpx<T> v[First::VALS];
    First::read(v, lds, tid);
    __syncthreads();
    reg2reg(v, lds, tw, tid, out);
  }

  // Final outputs from registers to LDS in natural order (no barrier).
  __device__ __forceinline__ static void store_last(const cpx<T>* out, cpx<T>* lds, int tid) {
    Last::write(out, lds, tid);
  }
};

}  // namespace hfx
