// Natural logarithm of the bulk chemical potentials (Eqs. 15-21 each take one
// or two logarithms per node per step).
//
// Method: reduce x = 2^e m with m in [sqrt(1/2), sqrt(2)); then
// ln m = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 3 - 2 sqrt(2), summed as
// the Taylor series 2 (s + s^3/3 + s^5/5 + ... + s^19/19): the first omitted
// term is below 2^-55 of the sum.  ln x = e ln2 + ln m, with ln 2 carried as
// two doubles.  m - 1 is exact in this range, so results near x = 1 keep
// full relative accuracy.  The error stays within a few ulp; zero, negative,
// infinite and NaN arguments give what the C library gives (-inf, NaN, +inf,
// NaN).  Every rounding step is spelled out (fma, one division), so the host
// and device builds of this function return identical bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace cplbm {
namespace phys {

__host__ __device__ __forceinline__ double lnx(double x)
{
    constexpr double kSqrtHalf = 0.70710678118654752440;
    constexpr double kLn2Hi = 0.69314718055994530942;        // nearest double to ln 2
    constexpr double kLn2Lo = 2.3190468138462996154e-17;     // ln 2 - kLn2Hi
    int e = 0;
    double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1) for finite x > 0
    if (m < kSqrtHalf) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    // sum_{k>=1} z^(k-1) / (2k + 1), k = 1 ... 9
    double t = 1.0 / 19.0;
    t = fma(t, z, 1.0 / 17.0);
    t = fma(t, z, 1.0 / 15.0);
    t = fma(t, z, 1.0 / 13.0);
    t = fma(t, z, 1.0 / 11.0);
    t = fma(t, z, 1.0 / 9.0);
    t = fma(t, z, 1.0 / 7.0);
    t = fma(t, z, 1.0 / 5.0);
    t = fma(t, z, 1.0 / 3.0);
    const double lm = 2.0 * fma(s * z, t, s);  // ln m
    const double de = (double)e;
    const double r = fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
    if (x > 0.0) return x < INFINITY ? r : x;
    return x == 0.0 ? -INFINITY : NAN;
}

}  // namespace phys
}  // namespace cplbm
