// Host-side construction of Stockham stage twiddle tables.
//
// For a radix schedule (R_0, ..., R_{S-1}) the table lists, for every stage
// with span Ns > 1 (Ns = R_0 ... R_{s-1}), the factors W_{Ns R}^{r k}
// = exp(-2 pi i r k / (Ns R)) for k = 0..Ns-1, r = 1..R-1, at index
// k*(R-1) + r-1 after the entries of the earlier stages.  Values are
// evaluated in float64 and rounded once to the working precision.
#pragma once

#include <vector>

#include "trig.hpp"

namespace hfx {

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
