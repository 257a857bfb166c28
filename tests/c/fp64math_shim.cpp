// Host build of the FP64 pair sweeps' exp(-x) (pb_fp64math.h) as a C function,
// for comparing the device's results with it bit for bit.  Built with
// -ffp-contract=off so that only the header's explicit fused multiply-adds
// are fused.
#include <cstdint>

#define PB_HD inline
#include "pb_fp64math.h"

extern "C" void host_exp_neg_pair(int64_t n, const double *x, double *out)
{
    for (int64_t k = 0; k < n; ++k)
        out[k] = pbk::fm::exp_neg_pair(x[k]);
}
