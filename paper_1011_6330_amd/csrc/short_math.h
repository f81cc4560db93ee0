// short_math.h -- short forms of the correctly rounded double division and
// square root: the operations of the general routines without their scaling
// and special-case steps, so the same bits wherever those steps do nothing.
//   nr_recip(d): the hardware reciprocal estimate and two Newton steps;
//   nr_div(n, d, nr_recip(d)) = n / d for |d| in [2^-300, 2^300] and n = 0 or
//     |n| in [2^-600, 2^400] (no operand scaling, no denormal quotient);
//   gs_sqrt(t) = sqrt(t) for finite t >= 2^-767 (Goldschmidt from the hardware
//     reciprocal square root estimate, then two residual corrections).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace pcpic {

__device__ __forceinline__ double nr_recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double nr_div(double n, double d, double r)
{
    const double q = n * r;
    const double rem = fma(-d, q, n);
    return fma(rem, r, q);
}
__device__ __forceinline__ double gs_sqrt(double t)
{
    const double y = __builtin_amdgcn_rsq(t);
    double g = t * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, t);
    g = fma(d, h, g);
    d = fma(-g, g, t);
    return fma(d, h, g);
}
// a dividend nr_div takes: 0 or a magnitude within [2^-600, 2^400]
__device__ __forceinline__ bool nr_num_ok(double n) { return n == 0.0 || (fabs(n) >= 0x1p-600 && fabs(n) <= 0x1p+400); }

}  // namespace pcpic
