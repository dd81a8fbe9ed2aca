// Device helpers shared by the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "rt_internal.h"

namespace rt {

constexpr double kFourPi = 12.566370614359172953850573533118;

// Cross-lane moves for the group sums below, on 32-bit halves.  DPP
// (quad_perm, row_half_mirror, row_mirror) stays inside a 16-lane row;
// v_permlane16_swap / v_permlane32_swap (gfx950) exchange rows 0<->1, 2<->3
// and the two wavefront halves.  Every lane of these row permutations reads
// a valid source lane and every row and bank is enabled, so no lane keeps
// the destination's old value and none needs to be set first.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u(unsigned x) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = dpp_u<CTRL>((unsigned)b), hi = dpp_u<CTRL>((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7-i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15-i within 16

// x of this lane plus x of the partner row (16 lanes apart) or half (32
// lanes apart); both partners form the same sum in the same order.
template <int DIST>
__device__ __forceinline__ double swap_add(double x) {
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    unsigned l0, l1, h0, h1;
    if constexpr (DIST == 16) {
        const auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = L[0]; l1 = L[1]; h0 = H[0]; h1 = H[1];
    } else {
        const auto L = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto H = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = L[0]; l1 = L[1]; h0 = H[0]; h1 = H[1];
    }
    const double a = __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0));
    const double c = __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
    return a + c;
}
template <int DIST>
__device__ __forceinline__ int swap_add_i(int x) {
    if constexpr (DIST == 16) {
        const auto L = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
        return (int)L[0] + (int)L[1];
    } else {
        const auto L = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
        return (int)L[0] + (int)L[1];
    }
}

// Sum over aligned groups of W lanes (W a power of two, 4 <= W <= 64); every
// lane of a group receives the same, bitwise identical, sum.
template <int W>
__device__ __forceinline__ double group_sum(double x) {
    static_assert(W >= 4 && W <= 64 && (W & (W - 1)) == 0, "group width");
    x += dpp_d<kDppXor1>(x);
    x += dpp_d<kDppXor2>(x);
    if constexpr (W >= 8) x += dpp_d<kDppHalfMirror>(x);
    if constexpr (W >= 16) x += dpp_d<kDppMirror>(x);
    if constexpr (W >= 32) x = swap_add<16>(x);
    if constexpr (W >= 64) x = swap_add<32>(x);
    return x;
}

// K independent sums over the same groups, step by step interleaved (each
// cross-lane move then reads a register written several instructions
// earlier, so no DPP hazard padding is needed).
template <int W, int K>
__device__ __forceinline__ void group_sum_v(double (&x)[K]) {
    static_assert(W >= 4 && W <= 64 && (W & (W - 1)) == 0, "group width");
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] += dpp_d<kDppXor1>(x[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] += dpp_d<kDppXor2>(x[k]);
    if constexpr (W >= 8) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] += dpp_d<kDppHalfMirror>(x[k]);
    }
    if constexpr (W >= 16) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] += dpp_d<kDppMirror>(x[k]);
    }
    if constexpr (W >= 32) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = swap_add<16>(x[k]);
    }
    if constexpr (W >= 64) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = swap_add<32>(x[k]);
    }
}

// Sums over aligned 32-lane groups of P pairs of values (x[2p], x[2p+1]) and
// of S single values, in fewer instructions than group_sum_v: one
// v_permlane16_swap of the pair leaves the first value's row-0 + row-1 sum in
// row 0 and the second's in row 1, so one register carries both through the
// four in-row levels; a swap of that register with itself then hands each
// lane of the group both totals.  Every lane of a group receives bitwise
// identical sums.
__device__ __forceinline__ void split_d(double x, unsigned &lo, unsigned &hi) {
    const unsigned long long b = __double_as_longlong(x);
    lo = (unsigned)b;
    hi = (unsigned)(b >> 32);
}
__device__ __forceinline__ double join_d(unsigned lo, unsigned hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int P, int S>
__device__ __forceinline__ void group_sum32_pairs(double (&x)[2 * P], double (&y)[S > 0 ? S : 1]) {
    double s[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        unsigned al, ah, bl, bh;
        split_d(x[2 * p], al, ah);
        split_d(x[2 * p + 1], bl, bh);
        // first operand's odd rows <-> second operand's even rows
        const auto L = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
        const auto H = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
        s[p] = join_d(L[0], H[0]) + join_d(L[1], H[1]);
    }
    constexpr int NS = S;
#pragma unroll
    for (int lvl = 0; lvl < 4; ++lvl) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (lvl == 0) s[p] += dpp_d<kDppXor1>(s[p]);
            if (lvl == 1) s[p] += dpp_d<kDppXor2>(s[p]);
            if (lvl == 2) s[p] += dpp_d<kDppHalfMirror>(s[p]);
            if (lvl == 3) s[p] += dpp_d<kDppMirror>(s[p]);
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (lvl == 0) y[k] += dpp_d<kDppXor1>(y[k]);
            if (lvl == 1) y[k] += dpp_d<kDppXor2>(y[k]);
            if (lvl == 2) y[k] += dpp_d<kDppHalfMirror>(y[k]);
            if (lvl == 3) y[k] += dpp_d<kDppMirror>(y[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) y[k] = swap_add<16>(y[k]);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        unsigned lo, hi;
        split_d(s[p], lo, hi);
        const auto L = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto H = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        x[2 * p] = join_d(L[0], H[0]);       // the total row 0 held
        x[2 * p + 1] = join_d(L[1], H[1]);   // the total row 1 held
    }
}

// Wavefront-wide (64-lane) sums of K values, four per register: a
// v_permlane32_swap of two values leaves each one's half-sum in its own
// wavefront half, a v_permlane16_swap of two such registers leaves the four
// row sums in the four rows; the four in-row levels then run on one register
// for four values, and two self-swaps (rows, then halves) hand every lane all
// four totals.  K is padded to a multiple of four with zeros.  Every lane
// receives bitwise identical sums.
__device__ __forceinline__ void swap_pair(int dist, double a, double b, double &ra, double &rb) {
    unsigned al, ah, bl, bh;
    split_d(a, al, ah);
    split_d(b, bl, bh);
    if (dist == 16) {
        const auto L = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
        const auto H = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
        ra = join_d(L[0], H[0]);
        rb = join_d(L[1], H[1]);
    } else {
        const auto L = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
        const auto H = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
        ra = join_d(L[0], H[0]);
        rb = join_d(L[1], H[1]);
    }
}
template <int K>
__device__ __forceinline__ void wave_sum_quads(double (&x)[K]) {
    constexpr int Q = (K + 3) / 4;
    double t[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = 4 * q + j < K ? x[4 * q + j] : 0.0;
        double a0, a1, b0, b1;
        swap_pair(32, v[0], v[1], a0, a1);   // half 0: v0, half 1: v1
        swap_pair(32, v[2], v[3], b0, b1);   // half 0: v2, half 1: v3
        const double s01 = a0 + a1, s23 = b0 + b1;
        double c0, c1;
        swap_pair(16, s01, s23, c0, c1);     // rows 0..3: v0, v2, v1, v3
        t[q] = c0 + c1;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) t[q] += dpp_d<kDppXor1>(t[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q) t[q] += dpp_d<kDppXor2>(t[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q) t[q] += dpp_d<kDppHalfMirror>(t[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q) t[q] += dpp_d<kDppMirror>(t[q]);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double e, o;
        swap_pair(16, t[q], t[q], e, o);     // e: rows 0/2 (v0 | v1), o: rows 1/3 (v2 | v3)
        double r[4];
        swap_pair(32, e, e, r[0], r[1]);
        swap_pair(32, o, o, r[2], r[3]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (4 * q + j < K) x[4 * q + j] = r[j];
    }
}

template <int W>
__device__ __forceinline__ int group_sum_i(int x) {
    static_assert(W >= 4 && W <= 64 && (W & (W - 1)) == 0, "group width");
    x += (int)dpp_u<kDppXor1>((unsigned)x);
    x += (int)dpp_u<kDppXor2>((unsigned)x);
    if constexpr (W >= 8) x += (int)dpp_u<kDppHalfMirror>((unsigned)x);
    if constexpr (W >= 16) x += (int)dpp_u<kDppMirror>((unsigned)x);
    if constexpr (W >= 32) x = swap_add_i<16>(x);
    if constexpr (W >= 64) x = swap_add_i<32>(x);
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

// a / b: in FP32 with the hardware reciprocal (about 1 ulp), in FP64 an
// IEEE division
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double quot(double a, double b) { return a / b; }

// Positive root of B4 T^4 + B1 T + B0 (Sec. 2.5) by Newton's method started
// at T_hi = min(-B0/B1, (-B0/B4)^(1/4)) >= root: the polynomial is
// increasing and convex on T >= 0, so the iterates decrease monotonically to
// the root; stop when they no longer decrease.  No positive root (B0 >= 0 or
// a non-finite coefficient): 1e-12 and bad = 1.
// A root that over- or underflowed (coefficients near the ends of the double
// range) counts as no usable root: the floor, like the other failures.
__device__ __forceinline__ double root_or_floor(double T, int &bad) {
    if (T > 0.0 && T < 1e300) return T;
    bad = 1;
    return 1e-12;
}

__device__ __forceinline__ double quartic_root(double B4, double B1, double B0, int &bad) {
    bad = 0;
    if (!(isfinite(B4) && isfinite(B1) && isfinite(B0)) || !(B0 < 0.0) || !(B1 > 0.0)) {
        bad = 1;
        return 1e-12;
    }
    const double lin = -B0 / B1;
    if (!(B4 > 0.0)) return root_or_floor(lin, bad);
    double T = fmin(lin, sqrt(sqrt(-B0 / B4)));
    for (int it = 0; it < 200; ++it) {
        const double T3 = T * T * T;
        const double p = B4 * T3 * T + B1 * T + B0;
        const double dp = 4.0 * B4 * T3 + B1;
        const double Tn = T - p / dp;
        if (!(Tn < T)) break;
        T = Tn;
    }
    return root_or_floor(T, bad);
}

// Same root, fewer instructions: Newton steps use a refined reciprocal, and
// the fourth-root bound starts from an FP32 estimate enlarged by 1e-5 (still
// an upper bound, so the iteration stays monotone).  A hint h (the gas
// temperature before the step) gives a closer upper bound: h itself when
// P(h) >= 0, else one Newton step from h, which lands above the root because
// P is convex and increasing on T >= 0; the smaller of that and the bound
// above starts the iteration.  Agrees with quartic_root to a few ulp.
__device__ __forceinline__ double quartic_root_fast(double B4, double B1, double B0, int &bad,
                                                    double hint = 0.0) {
    bad = 0;
    if (!(isfinite(B4) && isfinite(B1) && isfinite(B0)) || !(B0 < 0.0) || !(B1 > 0.0)) {
        bad = 1;
        return 1e-12;
    }
    const double lin = -B0 * rcp64(B1);
    if (!(B4 > 0.0)) return root_or_floor(-B0 / B1, bad);
    const double x = -B0 * rcp64(B4);
    double T = lin;
    if (x < 1e30 && x > 1e-30) {
        const float q = sqrtf(sqrtf((float)x)) * 1.00001f;
        T = fmin(lin, (double)q);
    }
    if (hint > 0.0 && hint < T) {
        const double h3 = hint * hint * hint;
        const double ph = fma(B4 * h3, hint, fma(B1, hint, B0));
        const double th = ph >= 0.0 ? hint : hint - ph * rcp64(fma(4.0 * B4, h3, B1));
        T = fmin(T, th);
    }
    for (int it = 0; it < 200; ++it) {
        const double T3 = T * T * T;
        const double p = fma(B4 * T3, T, fma(B1, T, B0));
        const double dp = fma(4.0 * B4, T3, B1);
        const double Tn = T - p * rcp64(dp);
        if (!(Tn < T)) break;
        T = Tn;
    }
    return root_or_floor(T, bad);
}

// Radiation-dominated velocity substitute (Sec. 2.5), per cell, from the
// transport result's angle sums with the gas velocity u (sv: E = sum I nb^2
// dOm, R^00 = sum I dOm, R^0a = sum n^a I dOm and sum n^a nb I dOm, with
// nb = u0 - u.n): where E > rho + u_gas and the radiation velocity
// v = R^0a/R^00 is subluminal, each component of u moves toward the
// radiation's four-velocity by the fraction of the gap that one step of the
// coupling force closes, clamped to [0, 1]; u0 is recomputed.  Shared by the
// general and column kernels.
__device__ __forceinline__ void velocity_substitute(const double (&sv)[8], double rh, double Tm,
                                                    double aa, double as, double n0, double dt,
                                                    double cv, double kb, double a_rad,
                                                    double &u0, double &u1, double &u2,
                                                    double &u3) {
    const double ug = rh * cv * Tm;
    if (!(sv[1] > 0.0 && sv[0] > rh + ug)) return;
    const double iR = 1.0 / sv[1];
    const double vr[3] = {sv[2] * iR, sv[3] * iR, sv[4] * iR};
    const double v2 = vr[0] * vr[0] + vr[1] * vr[1] + vr[2] * vr[2];
    if (!(v2 < 1.0)) return;
    const double ur0 = 1.0 / sqrt(1.0 - v2);
    const double wg = rh + ug + rh * kb * Tm;
    const double Tm2 = Tm * Tm;
    const double emit = aa * a_rad * Tm2 * Tm2 + as * sv[0];
    const double uo[3] = {u1, u2, u3};
    double un[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double ura = ur0 * vr[a];
        const double Ga = -emit * uo[a] + (aa + as) * sv[5 + a];
        const double den = n0 * (wg * ur0 * ura - wg * u0 * uo[a]);
        double f = den != 0.0 ? Ga * dt / den : 0.0;
        f = fmin(fmax(f, 0.0), 1.0);
        un[a] = (1.0 - f) * uo[a] + f * ura;
    }
    u1 = un[0];
    u2 = un[1];
    u3 = un[2];
    u0 = sqrt(fma(u1, u1, fma(u2, u2, fma(u3, u3, 1.0))));
}

}  // namespace rt
