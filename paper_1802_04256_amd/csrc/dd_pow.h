// Correctly rounded x^q on gfx950 by double-double arithmetic.
//
// The radial basis R = (s + C^2)^q of the moment matrix is evaluated to
// ~2^-98 relative accuracy in double-double (the error-free transformations
// of Dekker 1971 and Knuth, TAOCP vol. 2 sec. 4.2.2: TwoSum, FastTwoSum,
// TwoProd via fma), then rounded once to double.  Because the double-double
// value is accurate far beyond the 2^-53 rounding step, that single rounding
// yields the correctly rounded power unless the exact value lies within
// 2^-95 relative of a midpoint between doubles; such a case is flagged so it
// can never pass silently (probability ~2^-42 per call).
//
//   log t : one Newton step y1 = y0 + (t * exp(-y0) - 1) from y0 = log(t)
//   exp z : z = k ln2 + r, r scaled by 2^-5, Taylor series to r^14/14!,
//           five doublings e^{2r} - 1 = s (s + 2), then * 2^k.
//   t^q   : exp(q * log t).
#pragma once

#include <hip/hip_runtime.h>

namespace rpim {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ dd fast_two_sum(double a, double b) {  // |a| >= |b|
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return {p, e};
}

__device__ __forceinline__ dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_mul(dd x, dd y) {
  dd p = two_prod(x.hi, y.hi);
  p.lo = __builtin_fma(x.hi, y.lo, __builtin_fma(x.lo, y.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_mul_d(dd x, double d) {
  dd p = two_prod(x.hi, d);
  p.lo = __builtin_fma(x.lo, d, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

// 1/n! for n = 2..14 as double-double (exact rationals rounded twice).
__constant__ static const double kInvFact[13][2] = {
    {0x1.0000000000000p-1, 0x0.0p+0},                  // 1/2!
    {0x1.5555555555555p-3, 0x1.5555555555555p-57},     // 1/3!
    {0x1.5555555555555p-5, 0x1.5555555555555p-59},     // 1/4!
    {0x1.1111111111111p-7, 0x1.1111111111111p-63},     // 1/5!
    {0x1.6c16c16c16c17p-10, -0x1.f49f49f49f49fp-65},   // 1/6!
    {0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-73},    // 1/7!
    {0x1.a01a01a01a01ap-16, 0x1.a01a01a01a01ap-76},    // 1/8!
    {0x1.71de3a556c734p-19, -0x1.c154f8ddc6c00p-73},   // 1/9!
    {0x1.27e4fb7789f5cp-22, 0x1.cbbc05b4fa99ap-76},    // 1/10!
    {0x1.ae64567f544e4p-26, -0x1.c062e06d1f209p-80},   // 1/11!
    {0x1.1eed8eff8d898p-29, -0x1.2aec959e14c06p-83},   // 1/12!
    {0x1.6124613a86d09p-33, 0x1.f28e0cc748ebep-87},    // 1/13!
    {0x1.93974a8c07c9dp-37, 0x1.05d6f8a2efd1fp-92},    // 1/14!
};

// e^z for a double-double z with |z| < 700.
__device__ __forceinline__ dd dd_exp(dd z) {
  const double ln2_hi = 0x1.62e42fefa39efp-1;
  const double ln2_lo = 0x1.abc9e3b39803fp-56;
  const double k = __builtin_rint(z.hi * 0x1.71547652b82fep+0);  // z / ln2, rounded
  dd r = dd_add(z, dd_mul_d(dd{-ln2_hi, -ln2_lo}, k));
  r.hi *= 0x1p-5;
  r.lo *= 0x1p-5;
  // expm1(r) = r + r^2/2! + ... + r^14/14!  (Horner in double-double)
  dd s = dd{kInvFact[12][0], kInvFact[12][1]};
  for (int i = 11; i >= 0; --i) {
    s = dd_mul(s, r);
    s = dd_add(s, dd{kInvFact[i][0], kInvFact[i][1]});
  }
  s = dd_mul(s, r);
  s = dd_add(s, dd{1.0, 0.0});
  s = dd_mul(s, r);
  // five doublings: expm1(2r) = expm1(r) * (expm1(r) + 2)
  for (int i = 0; i < 5; ++i) s = dd_mul(s, dd_add(s, dd{2.0, 0.0}));
  dd e = dd_add(s, dd{1.0, 0.0});
  const double scale = __builtin_ldexp(1.0, (int)k);
  return dd{e.hi * scale, e.lo * scale};
}

// log t for a double t > 0 as double-double.
__device__ __forceinline__ dd dd_log(double t) {
  const double y0 = ::log(t);
  dd u = dd_mul_d(dd_exp(dd{-y0, 0.0}), t);  // = exp(log t - y0) ~ 1
  dd d = two_sum(u.hi - 1.0, u.lo);           // u.hi - 1 is exact
  return dd_add(dd{y0, 0.0}, d);
}

// Correctly rounded t^q for t > 0.  *hard is set when the double-double value
// is too close to a rounding boundary for its error bound.
__device__ __forceinline__ double pow_cr(double t, double q, bool* hard) {
  dd y = dd_exp(dd_mul_d(dd_log(t), q));
  dd r = fast_two_sum(y.hi, y.lo);  // r.hi = round-to-nearest of hi + lo
  const double toward = r.lo >= 0.0 ? __builtin_inf() : -__builtin_inf();
  const double nb = ::nextafter(r.hi, toward);
  const double half = 0.5 * __builtin_fabs(nb - r.hi);
  if (half - __builtin_fabs(r.lo) <= 0x1p-95 * __builtin_fabs(r.hi)) *hard = true;
  return r.hi;
}

}  // namespace rpim
