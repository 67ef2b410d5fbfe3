// The objective over datasets of one n-plet: the mean of its D values, or the paired effect size
// between two conditions (Discussion: functions of the measures optimised across datasets).
#pragma once

#include "thoi_internal.hpp"

namespace thoi {

// v[d * B + b], d = 0..D-1.  MEAN: summed in ascending d.  PAIRED_EFFECT: x_p = v[p] - v[P + p]
// (D = 2P), mean(x) / sd(x) with sd on P - 1 degrees of freedom, NaN when sd = 0.  A NaN among
// the values gives NaN.
template <typename VT>
__device__ __forceinline__ double objective_of(const VT* __restrict__ v, int64_t D, int64_t B, int64_t b, int kind)
{
    if (kind == THOI_OBJ_MEAN) {
        double s = 0.0;
        for (int64_t d = 0; d < D; ++d) s += (double)v[d * B + b];
        return s / (double)D;
    }
    // paired effect size: x_p = v[p] - v[P + p], mean / sd (P - 1 degrees of freedom)
    const int64_t P = D / 2;
    double s = 0.0;
    for (int64_t p = 0; p < P; ++p) s += (double)v[p * B + b] - (double)v[(P + p) * B + b];
    const double m = s / (double)P;
    double q = 0.0;
    for (int64_t p = 0; p < P; ++p) {
        const double x = (double)v[p * B + b] - (double)v[(P + p) * B + b] - m;
        q += x * x;
    }
    const double sd = sqrt(q / (double)(P - 1));
    return sd > 0.0 ? m / sd : __builtin_nan("");
}

}  // namespace thoi
