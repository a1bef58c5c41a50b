// Compile-time and host-side cosine/sine of rational angles 2*pi*p/q in float64.
//
// Used for the FFT twiddle factors: constants inside the radix codelets are
// folded at compile time, and the per-stage twiddle tables are evaluated on
// the host in float64 and rounded once to the working precision.
//
// Method: exact octant reduction on the integers (8p mod 8q), then Taylor
// series of sin and cos on [0, pi/4] summed to 27th order (truncation error
// below 1e-30 there), so the only rounding is in the final sums.
#pragma once

namespace hfx {

struct SinCos {
  double c, s;
};

__host__ __device__ constexpr double taylor_sin(double x) {
  // sum_{k>=0} (-1)^k x^(2k+1) / (2k+1)!
  double term = x, sum = x;
  for (int k = 1; k <= 13; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

__host__ __device__ constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k <= 13; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

// cos and sin of 2*pi*p/q for integers p (any sign), q > 0.
__host__ __device__ constexpr SinCos sincos_2pi(long long p, long long q) {
  constexpr double kPi4 = 0.78539816339744830961566084581987572;  // pi/4
  long long a = (8 * p) % (8 * q);
  if (a < 0) a += 8 * q;
  // angle = (pi/4) * a / q with a / q in [0, 8)
  long long o = a / q;          // octant 0..7
  long long rem = a - o * q;    // angle within the octant = (pi/4) rem / q
  double phi = 0.0, S = 0.0, C = 0.0;
  if ((o & 1) == 0) {
    phi = kPi4 * (double)rem / (double)q;
  } else {
    phi = kPi4 * (double)(q - rem) / (double)q;
  }
  S = taylor_sin(phi);
  C = taylor_cos(phi);
  switch (o) {
    case 0: return {C, S};
    case 1: return {S, C};
    case 2: return {-S, C};
    case 3: return {-C, S};
    case 4: return {-C, -S};
    case 5: return {-S, -C};
    case 6: return {S, -C};
    default: return {C, -S};
  }
}

}  // namespace hfx
