// Host-side construction of Stockham stage twiddle tables.
//
// For a radix schedule (R_0, ..., R_{S-1}) the table lists, for every stage
// with span Ns > 1 (Ns = R_0 ... R_{s-1}), the factors W_{Ns R}^{r k}
// = exp(-2 pi i r k / (Ns R)) for k = 0..Ns-1, r = 1..R-1, at index
// k*(R-1) + r-1 after the entries of the earlier stages.  Values are
// evaluated in float64 and rounded once to the working precision.
#pragma once

#include <cmath>
#include <vector>

#include "trig.hpp"

namespace hfx {

// float32 representation of a unit complex number: among the float32
// neighbours (within two units in the last place) of cos and sin, the pair
// whose norm c^2 + s^2 is closest to 1 (ties: smaller angle error).  A norm
// error scales every value passing through the twiddle and, being one-sided
// for plain rounding, biases transform energies; an angle error keeps the
// transform unitary.
inline void unit_f32(double c, double s, float* cf, float* sf) {
  const float c0 = (float)c, s0 = (float)s;
  float bc = c0, bs = s0;
  double best_norm = 1e300, best_ang = 1e300;
  const double ang = std::atan2(s, c);
  auto step = [](float x, int d) {
    for (; d > 0; --d) x = std::nextafter(x, 2.0f);
    for (; d < 0; ++d) x = std::nextafter(x, -2.0f);
    return x;
  };
  for (int dc = -2; dc <= 2; ++dc)
    for (int ds = -2; ds <= 2; ++ds) {
      const float ct = step(c0, dc), st = step(s0, ds);
      const double nrm = std::fabs((double)ct * ct + (double)st * st - 1.0);
      double da = std::fabs(std::atan2((double)st, (double)ct) - ang);
      if (da > 3.14159265358979323846) da = 2 * 3.14159265358979323846 - da;
      if (nrm < best_norm || (nrm == best_norm && da < best_ang)) {
        best_norm = nrm;
        best_ang = da;
        bc = ct;
        bs = st;
      }
    }
  *cf = bc;
  *sf = bs;
}

inline std::vector<double> twiddle_table(const int* radices, int count) {
  std::vector<double> out;  // interleaved (re, im)
  long long ns = 1;
  for (int s = 0; s < count; ++s) {
    const int r_s = radices[s];
    if (ns > 1) {
      for (long long k = 0; k < ns; ++k) {
        for (int r = 1; r < r_s; ++r) {
          const SinCos w = sincos_2pi(-(long long)r * k, ns * r_s);
          out.push_back(w.c);
          out.push_back(w.s);
        }
      }
    }
    ns *= r_s;
  }
  return out;
}

}  // namespace hfx
