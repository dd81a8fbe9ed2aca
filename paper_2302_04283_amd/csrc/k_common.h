// Device helpers shared by the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "rt_internal.h"

namespace rt {

constexpr double kFourPi = 12.566370614359172953850573533118;

// Sum over aligned groups of W lanes (W a power of two <= 64).
template <int W>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

template <int W>
__device__ __forceinline__ int group_sum_i(int x) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// 1/x in FP64: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// 1/x in FP64 with one Newton step on the hardware estimate (the estimate's
// error is squared, which suffices when it is below ~2^-26).
__device__ __forceinline__ double rcp64_1(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// Half of the van Leer (1974) harmonic-mean slope of the three values
// (a, b, c) in index space: delta/2 = (b-a)(c-b)/((b-a)+(c-b)) when the two
// differences share a sign, else 0 (Sec. 2.3, PLM).
__device__ __forceinline__ float half_slope(float a, float b, float c) {
    const float dm = b - a, dp = c - b;
    const float prod = dm * dp;
    return prod > 0.0f ? prod * __builtin_amdgcn_rcpf(dm + dp) : 0.0f;
}
__device__ __forceinline__ double half_slope(double a, double b, double c) {
    const double dm = b - a, dp = c - b;
    const double prod = dm * dp;
    return prod > 0.0 ? (2.0 * prod) / (dm + dp) * 0.5 : 0.0;
}

// Positive root of B4 T^4 + B1 T + B0 (Sec. 2.5) by Newton's method started
// at T_hi = min(-B0/B1, (-B0/B4)^(1/4)) >= root: the polynomial is
// increasing and convex on T >= 0, so the iterates decrease monotonically to
// the root; stop when they no longer decrease.  No positive root (B0 >= 0 or
// a non-finite coefficient): 1e-12 and bad = 1.
__device__ __forceinline__ double quartic_root(double B4, double B1, double B0, int &bad) {
    bad = 0;
    if (!(isfinite(B4) && isfinite(B1) && isfinite(B0)) || !(B0 < 0.0) || !(B1 > 0.0)) {
        bad = 1;
        return 1e-12;
    }
    const double lin = -B0 / B1;
    if (!(B4 > 0.0)) return lin;
    double T = fmin(lin, sqrt(sqrt(-B0 / B4)));
    for (int it = 0; it < 200; ++it) {
        const double T3 = T * T * T;
        const double p = B4 * T3 * T + B1 * T + B0;
        const double dp = 4.0 * B4 * T3 + B1;
        const double Tn = T - p / dp;
        if (!(Tn < T)) break;
        T = Tn;
    }
    return T;
}

// Same root, fewer instructions: Newton steps use a refined reciprocal, and
// the fourth-root bound starts from an FP32 estimate enlarged by 1e-5 (still
// an upper bound, so the iteration stays monotone).  Agrees with
// quartic_root to a few ulp.
__device__ __forceinline__ double quartic_root_fast(double B4, double B1, double B0, int &bad) {
    bad = 0;
    if (!(isfinite(B4) && isfinite(B1) && isfinite(B0)) || !(B0 < 0.0) || !(B1 > 0.0)) {
        bad = 1;
        return 1e-12;
    }
    const double lin = -B0 * rcp64(B1);
    if (!(B4 > 0.0)) return -B0 / B1;
    const double x = -B0 * rcp64(B4);
    double T = lin;
    if (x < 1e30 && x > 1e-30) {
        const float q = sqrtf(sqrtf((float)x)) * 1.00001f;
        T = fmin(lin, (double)q);
    }
    for (int it = 0; it < 200; ++it) {
        const double T3 = T * T * T;
        const double p = fma(B4 * T3, T, fma(B1, T, B0));
        const double dp = fma(4.0 * B4, T3, B1);
        const double Tn = T - p * rcp64(dp);
        if (!(Tn < T)) break;
        T = Tn;
    }
    return T;
}

}  // namespace rt
