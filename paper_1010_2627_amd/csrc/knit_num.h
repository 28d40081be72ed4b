// Scalar and complex arithmetic for the device code: float, double and
// double-double ("dd", an unevaluated sum hi + lo of two doubles, about 106
// significant bits; error-free transformations of Knuth and Dekker, as
// collected by Hida, Li and Bailey, "Algorithms for quad-double precision
// floating point arithmetic", ARITH-15, 2001).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knit {

// The error-free transformations below are exact only if every product and
// sum is rounded on its own; HIP compiles with FP contraction enabled across
// statements, which would fuse e.g. the product of two_prod into the sum of
// quick_two_sum.  Contraction is therefore off for the double-double code.
#pragma clang fp contract(off)

struct dd {
  double hi, lo;
};

// ---------------------------------------------------------------- error-free transformations
__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {  // requires |a| >= |b|
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return {p, e};
}

// ---------------------------------------------------------------- real ops, overloaded per type
__device__ __forceinline__ float r_add(float a, float b) { return a + b; }
__device__ __forceinline__ double r_add(double a, double b) { return a + b; }
__device__ __forceinline__ dd r_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ float r_neg(float a) { return -a; }
__device__ __forceinline__ double r_neg(double a) { return -a; }
__device__ __forceinline__ dd r_neg(dd a) { return {-a.hi, -a.lo}; }
template <class R> __device__ __forceinline__ R r_sub(R a, R b) { return r_add(a, r_neg(b)); }

__device__ __forceinline__ float r_mul(float a, float b) { return a * b; }
__device__ __forceinline__ double r_mul(double a, double b) { return a * b; }
__device__ __forceinline__ dd r_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}
// c + a*b
__device__ __forceinline__ float r_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double r_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ dd r_fma(dd a, dd b, dd c) { return r_add(c, r_mul(a, b)); }

__device__ __forceinline__ float r_div(float a, float b) { return a / b; }
__device__ __forceinline__ double r_div(double a, double b) { return a / b; }
__device__ __forceinline__ dd r_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = r_sub(a, r_mul(b, dd{q1, 0.0}));
  double q2 = r.hi / b.hi;
  r = r_sub(r, r_mul(b, dd{q2, 0.0}));
  double q3 = r.hi / b.hi;
  dd q = quick_two_sum(q1, q2);
  return r_add(q, dd{q3, 0.0});
}

#pragma clang fp contract(fast)

// leading part, used for magnitudes and pivot choice
__device__ __forceinline__ double r_lead(float a) { return (double)a; }
__device__ __forceinline__ double r_lead(double a) { return a; }
__device__ __forceinline__ double r_lead(dd a) { return a.hi; }

template <class R> __device__ __forceinline__ R r_from(double x);
template <> __device__ __forceinline__ float r_from<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ double r_from<double>(double x) { return x; }
template <> __device__ __forceinline__ dd r_from<dd>(double x) { return dd{x, 0.0}; }

__device__ __forceinline__ double r_to_double(float a) { return (double)a; }
__device__ __forceinline__ double r_to_double(double a) { return a; }
__device__ __forceinline__ double r_to_double(dd a) { return a.hi + a.lo; }

// ---------------------------------------------------------------- complex
template <class R>
struct cpx {
  R re, im;
};

template <class R> __device__ __forceinline__ cpx<R> c_make(R re, R im) { return {re, im}; }
template <class R> __device__ __forceinline__ cpx<R> c_zero() { return {r_from<R>(0.0), r_from<R>(0.0)}; }
template <class R> __device__ __forceinline__ cpx<R> c_one() { return {r_from<R>(1.0), r_from<R>(0.0)}; }
template <class R> __device__ __forceinline__ cpx<R> c_add(cpx<R> a, cpx<R> b) {
  return {r_add(a.re, b.re), r_add(a.im, b.im)};
}
template <class R> __device__ __forceinline__ cpx<R> c_sub(cpx<R> a, cpx<R> b) {
  return {r_sub(a.re, b.re), r_sub(a.im, b.im)};
}
template <class R> __device__ __forceinline__ cpx<R> c_neg(cpx<R> a) { return {r_neg(a.re), r_neg(a.im)}; }
template <class R> __device__ __forceinline__ cpx<R> c_conj(cpx<R> a) { return {a.re, r_neg(a.im)}; }
template <class R> __device__ __forceinline__ cpx<R> c_mul(cpx<R> a, cpx<R> b) {
  return {r_sub(r_mul(a.re, b.re), r_mul(a.im, b.im)), r_add(r_mul(a.re, b.im), r_mul(a.im, b.re))};
}
// c + a*b
template <class R> __device__ __forceinline__ cpx<R> c_fma(cpx<R> a, cpx<R> b, cpx<R> c) {
  R re = r_fma(a.re, b.re, c.re);
  re = r_fma(r_neg(a.im), b.im, re);
  R im = r_fma(a.re, b.im, c.im);
  im = r_fma(a.im, b.re, im);
  return {re, im};
}
// c - a*b
template <class R> __device__ __forceinline__ cpx<R> c_fms(cpx<R> a, cpx<R> b, cpx<R> c) {
  return c_fma(c_neg(a), b, c);
}
template <class R> __device__ __forceinline__ cpx<R> c_inv(cpx<R> a) {
  // 1/a = conj(a) / |a|^2, with a power-of-two prescale against overflow
  double m = fmax(fabs(r_lead(a.re)), fabs(r_lead(a.im)));
  int e = 0;
  if (m > 0.0 && m < 1e300) (void)frexp(m, &e);
  R s = r_from<R>(ldexp(1.0, -e));
  cpx<R> b = {r_mul(a.re, s), r_mul(a.im, s)};
  R den = r_add(r_mul(b.re, b.re), r_mul(b.im, b.im));
  R inv = r_div(r_from<R>(1.0), den);
  R f = r_mul(inv, s);
  return {r_mul(b.re, f), r_neg(r_mul(b.im, f))};
}
template <class R> __device__ __forceinline__ double c_abs1(cpx<R> a) {
  return fabs(r_lead(a.re)) + fabs(r_lead(a.im));
}
template <class R> __device__ __forceinline__ cpx<R> c_from(double re, double im) {
  return {r_from<R>(re), r_from<R>(im)};
}

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

}  // namespace knit
