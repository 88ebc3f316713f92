// Exponentials in base 2 for the annkin kernels, from a rounding reduction
// and the Taylor series of 2^f on |f| <= 1/2 (no device-library calls).
#pragma once
#include <hip/hip_runtime.h>

namespace ak {

// ln(2)^k / k!, the Taylor coefficients of 2^f = exp(f ln 2)
__device__ constexpr double kExp2Taylor[13] = {1.0,
                                              0.69314718055994530942,
                                              0.24022650695910071233,
                                              0.055504108664821579953,
                                              0.0096181291076284771620,
                                              0.0013333558146428443424,
                                              0.00015403530393381609954,
                                              0.000015252733804059840280,
                                              0.0000013215486790144309489,
                                              1.0178086009239699728e-7,
                                              7.0549116208011233099e-9,
                                              4.4455382718708114975e-10,
                                              2.5678435993488205142e-11};

// 2^g and 2^-g in double from one polynomial evaluation: g = n + f with n
// the nearest integer (|f| <= 1/2), 2^f = exp(f ln 2) by its Taylor series
// split into even and odd parts E(f) + O(f), so that 2^-f = E(f) - O(f).
// Degree 12 (error below one double ulp) or 10 (below 3e-13 relative).
template <int DEG>
__device__ __forceinline__ void exp2_pair(double g, double &pos, double &neg)
{
    const double n = __builtin_rint(g);
    const double f = g - n;
    const double f2 = f * f;
    double E = kExp2Taylor[DEG - (DEG & 1)];
#pragma unroll
    for (int k = DEG - (DEG & 1) - 2; k >= 0; k -= 2) E = __builtin_fma(E, f2, kExp2Taylor[k]);
    constexpr int top_odd = (DEG & 1) ? DEG : DEG - 1;
    double O = kExp2Taylor[top_odd];
#pragma unroll
    for (int k = top_odd - 2; k >= 1; k -= 2) O = __builtin_fma(O, f2, kExp2Taylor[k]);
    O *= f;
    const int ni = (int)n;
    pos = __builtin_ldexp(E + O, ni);
    neg = __builtin_ldexp(E - O, -ni);
}

// x * 2^t in double: t = n + f with n the nearest integer, 2^f by the
// degree-12 Taylor polynomial (error below two ulps), the power of two
// applied exactly by ldexp (which also gives the correct overflow to inf
// and underflow to 0).
__device__ __forceinline__ double scale_exp2(double x, double t)
{
    const double n = __builtin_rint(t);
    const double f = t - n;
    double p = kExp2Taylor[12];
#pragma unroll
    for (int k = 11; k >= 0; --k) p = __builtin_fma(p, f, kExp2Taylor[k]);
    return __builtin_ldexp(x * p, (int)n);
}

}  // namespace ak
