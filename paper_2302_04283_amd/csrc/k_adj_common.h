// Per-face arithmetic of the transport adjoint (Sec. 2.3-2.4 reversed),
// shared by the general gather (k_adjoint.hip) and the column march
// (k_adj_column.hip): both kernels form every term with these helpers, in
// the same order, so they give bit-identical results.
//
// The upwind PLM value of a face is V = I_u + sigma h(I_{u-1}, I_u, I_{u+1})
// with h(l, m, r) = (m-l)(r-m)/(r-l) half the van Leer slope (zero unless
// the two differences share a sign) and sigma = +1 when the motion along
// the axis is positive (upwind cell below the face), -1 otherwise.  Its
// partial derivatives, with a = m - l, b = r - m, x = a/(a+b), y = b/(a+b):
//   dh/dl = -y^2,  dh/dm = y^2 - x^2,  dh/dr = x^2.
// The branch test a*b > 0 is formed from the same two differences as the
// forward step's, so the adjoint differentiates the branch the forward took.
#pragma once

#include "k_transport.h"

namespace rt {

// 1/s: the hardware reciprocal in FP32, two Newton steps on it in FP64
template <typename Real>
__device__ __forceinline__ Real inv(Real s) {
    if constexpr (sizeof(Real) == 4)
        return __builtin_amdgcn_rcpf(s);
    else
        return rcp64(s);
}

// x^2 and y^2 of the limiter h(l, m, r) (both zero on the flat branch;
// formed on both branches and selected, so no divergent branch)
template <typename Real>
__device__ __forceinline__ void half_slope_partials(Real l, Real m, Real r, Real &hx, Real &hy) {
    const Real a = m - l, b = r - m;
    const Real i = inv(a + b);
    const Real x = a * i, y = b * i;
    const bool on = a * b > Real(0);
    hx = on ? x * x : Real(0);
    hy = on ? y * y : Real(0);
}

// dh_u / dI_x for the upwind cell u = -1, 0, +1 relative to x (x is the
// right, middle or left argument of h_u)
template <typename Real>
__device__ __forceinline__ Real dh_at(int u, Real hx, Real hy) {
    return u == 1 ? -hy : (u == 0 ? hy - hx : hx);
}

// dV / dI_x of a face: 1 if x is the upwind cell, plus sigma dh_u/dI_x
template <typename Real>
__device__ __forceinline__ Real face_weight(bool center, bool pos, bool plm, Real dh) {
    Real d = center ? Real(1) : Real(0);
    if (plm) d += pos ? dh : -dh;
    return d;
}

// dJ/dF of the face between cells b (below) and a (above): the face is the
// upper face of b and the lower face of a, Q*_a gains dt F / V_a and Q*_b
// loses dt F / V_b
template <typename Real>
__device__ __forceinline__ Real face_adjoint(Real dtR, Real psi_a, Real iv_a, Real psi_b, Real iv_b) {
    return dtR * (psi_a * iv_a - psi_b * iv_b);
}

// dJ/dF on the luminosity face: J = w dt sum dOmega (flux leaving through
// the upper face, or entering through the lower face)
template <typename Real>
__device__ __forceinline__ Real lum_seed(const DevGrid &G, double lum_weight, double dt, int n) {
    return Real((G.lum_side == 1 ? -1.0 : 1.0) * lum_weight * dt * G.domega[n]);
}

template <typename Real>
__device__ __forceinline__ void face_add(Real &lam, Real lF, Real C, Real d) {
    lam += lF * C * d;
}

// angular edge between directions lo and hi whose upwind side is the
// direction n itself: dJ/dI_n gains -dt w (psi_lo/dOmega_lo - psi_hi/dOmega_hi).
// Seen from n, with p the edge's other direction, that is
// s (psi_n/dOmega_n - psi_p/dOmega_p) with s = -dt w when n is the lower
// direction and +dt w when it is the upper one; 1/dOmega is rounded to the
// intensity precision.  edge_weight forms s; edge_add adds the term given
// a_n = psi_n/dOmega_n (one product for all of n's edges).  Both fused
// multiply-adds are written out, so every kernel rounds them alike.
template <typename Real>
__device__ __forceinline__ Real fmar(Real a, Real b, Real c) {
    if constexpr (sizeof(Real) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

template <typename Real>
__device__ __forceinline__ Real edge_weight(Real dtR, Real ww, bool n_is_lo) {
    const Real s = dtR * ww;
    return n_is_lo ? -s : s;
}

template <typename Real>
__device__ __forceinline__ void edge_add(Real &lam, Real a_n, Real psi_p, Real iom_p, Real s) {
    lam = fmar(fmar(-psi_p, iom_p, a_n), s, lam);
}

}  // namespace rt
