// Double-double arithmetic for the Gram matrices and Cholesky factors of
// the mixed-precision Cholesky QR.  Every function disables floating-point
// contraction in its body: the error-free transformations need every product
// and sum rounded separately (explicit fma() calls stay).
#pragma once

#include <hip/hip_runtime.h>

namespace tlr {

// Error-free transformations (Knuth TwoSum, FMA-based TwoProduct) and the
// double-double operations built on them (Dekker; Bailey's QD library).
struct dd {
  double hi, lo;
};
__device__ inline dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ inline dd two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ inline dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ inline dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
  const double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul(b, dd{q1, 0.0}));
  const double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul(b, dd{q2, 0.0}));
  const double q3 = r.hi / b.hi;
  const dd q = fast_two_sum(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}
__device__ inline dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
  if (!(a.hi > 0.0)) return {0.0, 0.0};
  const double x = 1.0 / sqrt(a.hi);
  const double ax = a.hi * x;
  const dd diff = dd_sub(a, two_prod(ax, ax));
  return fast_two_sum(ax, diff.hi * (x * 0.5));
}


// 1 / sqrt(a) for a > 0 to double-double accuracy: the FP64 estimate
// y0 = 1 / sqrt(a.hi) and one Newton step y1 = y0 + y0 (1 - a y0^2) / 2,
// with the residual 1 - a y0^2 formed in double-double.
__device__ inline dd dd_rsqrt(dd a) {
#pragma clang fp contract(off)
  const double y0 = 1.0 / sqrt(a.hi);
  const dd y2 = two_prod(y0, y0);
  const dd e = dd_sub(dd{1.0, 0.0}, dd_mul(a, y2));
  return fast_two_sum(y0, y0 * (e.hi * 0.5));
}

// 1 / a to double-double accuracy: y0 = 1 / a.hi and one Newton step, the
// residual 1 - a y0 formed with an FMA (exact for the high part).
__device__ inline dd dd_recip(dd a) {
#pragma clang fp contract(off)
  const double y0 = 1.0 / a.hi;
  const double r = fma(-a.hi, y0, 1.0) - a.lo * y0;
  return fast_two_sum(y0, y0 * r);
}

// a - b with the error bounded by about u^2 (|a| + |b|) (Dekker's add
// without the second error-free transformation of the low parts): enough
// where absolute accuracy against the operands is what counts.
__device__ inline dd dd_sub_sloppy(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = two_sum(a.hi, -b.hi);
  s.lo += a.lo - b.lo;
  return fast_two_sum(s.hi, s.lo);
}

// One step of the compensated dot product of Ogita, Rump and Oishi (Dot2):
// (s, c) accumulates x * y.
__device__ inline void dot2_step(double x, double y, double& s, double& c) {
#pragma clang fp contract(off)
  const double p = x * y;
  const double e = fma(x, y, -p);
  const double t = s + p;
  const double z = t - s;
  const double q = (s - (t - z)) + (p - z);
  s = t;
  c += q + e;
}

}  // namespace tlr
