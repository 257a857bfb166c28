// Host build of the library's FP64 pair-sweep functions (pb_fp64math.h):
// measures their error in units in the last place against long-double
// references.  Prints one "name value" line per statistic; the Python test
// (tests/test_fp64math_host.py) holds the bounds.
//   exp_neg_pair(x) against expl(-x) on [0, 708] (normal results) and the
//   subnormal/zero tail (708, 1e6];
//   rsqrt_refine(x, y0) against 1/sqrtl(x) for r^2 = x in [1e-8, 1e14], with
//   seeds y0 = (1 + d)/sqrt(x), |d| <= 2^-22 (twice the documented bound of
//   the hardware estimate).
#define PB_HD inline
#include "pb_fp64math.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>

using pbk::fm::exp_neg_pair;
using pbk::fm::EXP2_J256;
using pbk::fm::rsqrt_refine;

static long double ulp_of(long double v)
{
    // spacing of doubles at |v| (normal range)
    int e;
    std::frexp((double)v, &e);
    return std::ldexp(1.0L, e - 53);
}

int main()
{
    std::mt19937_64 rng(12345);
    // exp(-x), normal results
    double max_ulp_exp = 0.0, arg_max = 0.0;
    long double sum_ulp = 0.0L;
    int64_t n_exp = 0;
    auto probe = [&](double x) {
        const long double ref = expl(-(long double)x);
        const double y = exp_neg_pair(x);
        const double u = (double)(fabsl((long double)y - ref) / ulp_of(ref));
        sum_ulp += u;
        ++n_exp;
        if (u > max_ulp_exp) {
            max_ulp_exp = u;
            arg_max = x;
        }
    };
    for (int64_t k = 0; k <= 4000000; ++k)   // dense grid on [0, 708]
        probe(708.0 * (double)k / 4000000.0);
    std::uniform_real_distribution<double> small(0.0, 2.0), wide(0.0, 708.0);
    for (int k = 0; k < 2000000; ++k) {      // the range of near pairs, and all of it
        probe(small(rng));
        probe(wide(rng));
    }
    for (int k = 0; k < 200; ++k)            // tiny arguments, down to 1e-300
        probe(std::ldexp(1.0, -k * 5));
    std::printf("exp_max_ulp %.6f\n", max_ulp_exp);
    std::printf("exp_max_ulp_at %.17g\n", arg_max);
    std::printf("exp_mean_ulp %.6f\n", (double)(sum_ulp / n_exp));
    std::printf("exp_count %lld\n", (long long)n_exp);
    std::printf("exp_at_zero %.17g\n", exp_neg_pair(0.0));
    // tail: subnormal results and zero, never negative, NaN or inf
    double max_abs_tail = 0.0;
    int bad_tail = 0;
    for (int64_t k = 0; k <= 1000000; ++k) {
        const double x = 708.0 + (1e6 - 708.0) * std::pow((double)k / 1000000.0, 4.0);
        const double y = exp_neg_pair(x);
        if (!(y >= 0.0) || !std::isfinite(y))
            ++bad_tail;
        const long double ref = expl(-(long double)x);
        const double d = (double)fabsl((long double)y - ref);
        if (d > max_abs_tail)
            max_abs_tail = d;
    }
    std::printf("exp_tail_bad %d\n", bad_tail);
    std::printf("exp_tail_max_abs_in_min_subnormals %.6f\n", max_abs_tail / std::ldexp(1.0, -1074));
    std::printf("exp_beyond_745 %.17g\n", exp_neg_pair(745.2));
    std::printf("exp_at_max_arg %.17g\n", exp_neg_pair(5.8e6));
    // the table holds 2^(j/256) correctly rounded
    double max_tab_ulp = 0.0;
    for (int j = 0; j < 256; ++j) {
        const long double ref = exp2l((long double)j / 256.0L);
        const double u = (double)(fabsl((long double)EXP2_J256[j] - ref) / ulp_of(ref));
        if (u > max_tab_ulp)
            max_tab_ulp = u;
    }
    std::printf("table_max_ulp %.6f\n", max_tab_ulp);
    // rsqrt refinement
    double max_ulp_rsq = 0.0;
    std::uniform_real_distribution<double> lg(std::log(1e-8), std::log(1e14));
    std::uniform_real_distribution<double> dd(-1.0, 1.0);
    const double dmax = std::ldexp(1.0, -22);
    const double fixed[] = {0.0, dmax, -dmax, 0.5 * dmax, -0.5 * dmax};
    int64_t n_rsq = 0;
    for (int k = 0; k < 1000000; ++k) {
        const double x = std::exp(lg(rng));
        const long double ref = 1.0L / sqrtl((long double)x);
        for (int s = 0; s < 6; ++s) {
            const double d = s < 5 ? fixed[s] : dmax * dd(rng);
            const double y0 = (double)(ref * (1.0L + (long double)d));
            const double y = rsqrt_refine(x, y0);
            const double u = (double)(fabsl((long double)y - ref) / ulp_of(ref));
            if (u > max_ulp_rsq)
                max_ulp_rsq = u;
            ++n_rsq;
        }
    }
    std::printf("rsqrt_max_ulp %.6f\n", max_ulp_rsq);
    std::printf("rsqrt_count %lld\n", (long long)n_rsq);
    return 0;
}
