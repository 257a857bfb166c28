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

// 2^(j/32), j = 0..31, correctly rounded (the table of Tang's method).
constexpr double EXP2_J32[32] = {
    0x1.0000000000000p+0, 0x1.059b0d3158574p+0, 0x1.0b5586cf9890fp+0, 0x1.11301d0125b51p+0,
    0x1.172b83c7d517bp+0, 0x1.1d4873168b9aap+0, 0x1.2387a6e756238p+0, 0x1.29e9df51fdee1p+0,
    0x1.306fe0a31b715p+0, 0x1.371a7373aa9cbp+0, 0x1.3dea64c123422p+0, 0x1.44e086061892dp+0,
    0x1.4bfdad5362a27p+0, 0x1.5342b569d4f82p+0, 0x1.5ab07dd485429p+0, 0x1.6247eb03a5585p+0,
    0x1.6a09e667f3bcdp+0, 0x1.71f75e8ec5f74p+0, 0x1.7a11473eb0187p+0, 0x1.82589994cce13p+0,
    0x1.8ace5422aa0dbp+0, 0x1.93737b0cdc5e5p+0, 0x1.9c49182a3f090p+0, 0x1.a5503b23e255dp+0,
    0x1.ae89f995ad3adp+0, 0x1.b7f76f2fb5e47p+0, 0x1.c199bdd85529cp+0, 0x1.cb720dcef9069p+0,
    0x1.d5818dcfba487p+0, 0x1.dfc97337b9b5fp+0, 0x1.ea4afa2a490dap+0, 0x1.f50765b6e4540p+0,
};

// exp(-x) for 0 <= x < 4.6e7 (the reduced exponent must fit an int; with
// kappa <= 100 and coordinates within 1e5 of the origin, kappa r between real
// points stays below 3.5e7.  The sweeps' padding points, 2e6 out and of
// weight 0, reach larger arguments once kappa > 23; there the device's
// float-to-int conversion saturates, m = -2^26, and the result is 0) by
// Tang's table-driven method: with n = rint(-32 x / ln 2) =
// 32 m + j (j = n mod 32, m = floor(n / 32)), e^-x = 2^m 2^(j/32) e^r where
// r = -x - n ln2/32, |r| <= ln 2 / 64 (ln 2 / 32 split into a 32-bit head,
// exact times n while |n| < 2^21, and the rounded remainder).  e^r - 1 is
// r (1 + r/2 + ... + r^5/720) (truncation below 3.4e-18 relative), and the
// result 2^m (t + t (e^r - 1)) is rounded once from the table entry
// t = 2^(j/32): within 1.02 ulp of exp(-x) on [0, 708].  Beyond x = 708 the
// result is subnormal, beyond 745 it is 0; no overflow or special value can
// occur, so the general function's range checks are left out.
PB_HD double exp_neg_pair(double x)
{
    const double n = __builtin_rint(x * -46.16624130844683);   // <= 0
    const double r = fma(-n, 5.9631716539705866e-12, fma(-n, 0.02166084938653512, -x));
    const int ni = (int)n;
    double p = 1.3888888888888889e-03;        // 1/720
    p = fma(p, r, 8.3333333333333332e-03);    // 1/120
    p = fma(p, r, 4.1666666666666664e-02);    // 1/24
    p = fma(p, r, 1.6666666666666666e-01);    // 1/6
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    const double t = EXP2_J32[ni & 31];
    return ldexp(fma(t, p * r, t), ni >> 5);
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
