// dd.hpp -- double-double arithmetic on gfx950 (unevaluated sums hi + lo,
// |lo| <= ulp(hi)/2, about 106 bits).  Error-free transformations: the sum
// by Knuth's TwoSum, the product by one fused multiply-add (the exact
// residual of hi = fl(a b) is fma(a, b, -hi)).
//
// Every routine here switches floating-point contraction off (DD_EXACT):
// HIP contracts across statements by default, and would turn hi + lo, with
// hi = fl(a b), into fma(a, b, lo) -- the unrounded product in place of hi --
// which counts the rounding residual twice and leaves FP64 accuracy.
#pragma once
#include "common.hpp"

#define DD_EXACT _Pragma("clang fp contract(off)")

namespace msplit {

struct dd { double hi, lo; };
struct cdd { dd re, im; };

__device__ __forceinline__ dd two_sum(double a, double b)
{
    DD_EXACT
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) // |a| >= |b|
{
    DD_EXACT
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b)
{
    DD_EXACT
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    DD_EXACT
    dd s = two_sum(a.hi, b.hi);
    const dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { DD_EXACT return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { DD_EXACT return dd_add(a, dd_neg(b)); }
__device__ __forceinline__ dd dd_add_d(dd a, double b)
{
    DD_EXACT
    dd s = two_sum(a.hi, b);
    s.lo += a.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_mul(dd a, dd b)
{
    DD_EXACT
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b)
{
    DD_EXACT
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_sqr(dd a)
{
    DD_EXACT
    dd p = two_prod(a.hi, a.hi);
    p.lo += 2.0 * a.hi * a.lo;
    return quick_two_sum(p.hi, p.lo);
}

// (x + iy)^2 + c with c a double-double point
__device__ __forceinline__ cdd cdd_sqr_add(cdd z, cdd c)
{
    DD_EXACT
    const dd re = dd_add(dd_sub(dd_sqr(z.re), dd_sqr(z.im)), c.re);
    const dd xy = dd_mul(z.re, z.im);
    const dd im = dd_add({2.0 * xy.hi, 2.0 * xy.lo}, c.im);
    return {re, im};
}
__device__ __forceinline__ cdd cdd_sub(cdd a, cdd b) { DD_EXACT return {dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; }
__device__ __forceinline__ cdd cdd_neg(cdd a) { return {dd_neg(a.re), dd_neg(a.im)}; }
__device__ __forceinline__ double cdd_abs2_hi(cdd a) { DD_EXACT return a.re.hi * a.re.hi + a.im.hi * a.im.hi; }

} // namespace msplit
