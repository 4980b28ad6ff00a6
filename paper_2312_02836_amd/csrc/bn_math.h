// bn_math.h -- the FP64 natural logarithm of the burn kernels.
//
// The library logarithm handles every corner of the IEEE range at full
// generality and costs about a hundred instructions; the burn takes the
// logarithm of a temperature once per right-hand side and of error norms
// at every step-size decision, always of a positive finite number or of
// 0 / +inf.  This one is about forty instructions and stays within about
// one unit in the last place.
//
// Method (the classical artanh reduction): x = m 2^e with m in
// [sqrt(1/2), sqrt(2)).  With f = m - 1 (exact) and s = f / (2 + f),
// log m = 2 artanh s = 2s + s R(s^2),  R(z) = sum_{k>=1} 2 z^k / (2k + 1).
// With h = f^2 / 2, the identities 2s = f - s f and s f = h (1 - s) give
// log m = f - (h - s (h + R)), which keeps the rounding of the small
// correction away from the leading term f.
// |s| <= 3 - 2 sqrt(2) < 0.1716, so ten terms of R leave a truncation error
// below 1e-20 relative.  log x = e ln2 + log m, with ln 2 split into a head
// of 32 significant bits (e * head is exact) and a tail.
//
// The arithmetic is written out operation by operation (no contraction), so
// the host and the device evaluate it identically.
#pragma once

// (also compiled at run time with the generated kernels, where hiprtc
// provides the runtime and math declarations itself)
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <math.h>
#endif

namespace bn {

__host__ __device__ inline double bn_log(double x) {
#pragma clang fp contract(off)
  constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
  constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
  constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
  int e = 0;
  double m = frexp(x, &e);  // m in [1/2, 1) for positive finite x
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double p = 2.0 / 21.0;
  p = fma(p, z, 2.0 / 19.0);
  p = fma(p, z, 2.0 / 17.0);
  p = fma(p, z, 2.0 / 15.0);
  p = fma(p, z, 2.0 / 13.0);
  p = fma(p, z, 2.0 / 11.0);
  p = fma(p, z, 2.0 / 9.0);
  p = fma(p, z, 2.0 / 7.0);
  p = fma(p, z, 2.0 / 5.0);
  p = fma(p, z, 2.0 / 3.0);
  const double R = z * p;
  const double h = 0.5 * (f * f);
  const double ed = (double)e;
  // e ln2 + f - (h - (s (h + R) + e ln2_lo))
  const double c = h - fma(s, h + R, ed * kLn2Lo);
  double y = fma(ed, kLn2Hi, f - c);
  if (!(x > 0.0)) y = (x == 0.0) ? -__builtin_inf() : __builtin_nan("");
  if (x == __builtin_inf()) y = x;
  return y;
}

// x / d correctly rounded, given inv_d = 1 / d correctly rounded: the
// product q = x inv_d is within one unit in the last place of x / d, the
// remainder x - q d is exact in one fused multiply-add, and q + r inv_d then
// rounds to the correctly rounded quotient (Markstein's correction step)
// wherever that quotient is a normal number; a subnormal one may be off by
// one unit in its last place.  Three dependent operations instead of a full
// division, for a divisor that is fixed for a whole launch.  An infinite or
// NaN quotient is returned as the product gives it (inf / d = inf, NaN stays
// NaN).
__host__ __device__ inline double bn_div_by(double x, double d, double inv_d) {
  const double q = x * inv_d;
  const double r = fma(-q, d, x);
  const double c = fma(r, inv_d, q);
  return __builtin_isfinite(q) ? c : q;
}

}  // namespace bn
