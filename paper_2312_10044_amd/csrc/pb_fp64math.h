// FP64 elementary functions of the pair sweeps, specialised to the argument
// ranges a collocation pair produces.  They use only IEEE-754 operations that
// round the same way on the host and on the device (fused multiply-add,
// round-to-nearest-even, scaling by a power of two), so a host build of this
// header reproduces the device results bit for bit; the host build is what
// the accuracy tests run (they define PB_HD as plain `inline`).  Internal;
// not part of the public ABI.
#pragma once

#include <math.h>

#ifndef PB_HD
#define PB_HD __host__ __device__ __forceinline__
#endif

namespace pbk {
namespace fm {

// exp(-x) for 0 <= x < 1.4e9 (the reduced exponent must fit an int).
// Cody-Waite reduction: e^-x = 2^-n e^g with n = rint(x / ln 2) and
// g = n ln 2 - x, |g| <= ln 2 / 2, where ln 2 is split into a 32-bit head
// (n times it is exact while n < 2^21, i.e. x < 1.45e6) and the rounded
// remainder.  e^g is its Taylor series to degree 12 in Horner form, whose
// truncation error on that interval reaches 1.7e-16 relative (the first
// omitted term); with the roundings of the reduction and of the Horner steps
// the result is within 2.3 ulp of exp(-x) on [0, 708].  For
// 708 < x < 745 the result is subnormal, beyond 745 it is 0; no overflow or
// special value can occur, so the general function's range checks are left
// out.
PB_HD double exp_neg_pair(double x)
{
    const double n = __builtin_rint(x * 1.4426950408889634);
    const double g = fma(n, 1.9082149292705877e-10, fma(n, 0.6931471803691238, -x));
    double p = 2.08767569878681e-09;          // 1/12!
    p = fma(p, g, 2.505210838544172e-08);     // 1/11!
    p = fma(p, g, 2.755731922398589e-07);
    p = fma(p, g, 2.7557319223985893e-06);
    p = fma(p, g, 2.48015873015873e-05);
    p = fma(p, g, 0.0001984126984126984);
    p = fma(p, g, 0.001388888888888889);
    p = fma(p, g, 0.008333333333333333);
    p = fma(p, g, 0.041666666666666664);
    p = fma(p, g, 0.16666666666666666);
    p = fma(p, g, 0.5);
    p = fma(p, g, 1.0);
    p = fma(p, g, 1.0);
    return ldexp(p, -(int)n);
}

// 1/sqrt(x) for finite x > 0 from an estimate y of relative error eps:
// y (1 + e/2 + 3 e^2/8) with e = 1 - x y^2, the series of (1 - e)^(-1/2) to
// second order (one third-order Householder step).  The step leaves
// (5/16)(2 eps)^3 of the estimate's error; for the hardware estimate
// (eps <= 2^-22) that is far below the rounding of the step itself.
PB_HD double rsqrt_refine(double x, double y)
{
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

}  // namespace fm
}  // namespace pbk
