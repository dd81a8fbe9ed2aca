// Per-direction transport of the general step kernel (paper Sec. 2.3-2.4,
// 2.6), shared by the forward step and the adjoint (which recomputes I*).
#pragma once

#include "k_common.h"

namespace rt {

struct Cell {
    int i, j, k;     // cell coordinates
    long long c;     // linear cell index
    int gc;          // geometry cell index
};

__device__ __forceinline__ Cell make_cell(const DevGrid &G, long long c) {
    Cell x;
    x.c = c;
    x.i = (int)(c % G.n0);
    x.j = (int)((c / G.n0) % G.n1);
    x.k = (int)(c / ((long long)G.n0 * G.n1));
    x.gc = ((G.g2 > 1 ? x.k : 0) * G.g1 + (G.g1 > 1 ? x.j : 0)) * G.g0 + (G.g0 > 1 ? x.i : 0);
    return x;
}

__device__ __forceinline__ int face_geo(const DevGrid &G, int a, int fidx, const Cell &x) {
    const int xi = (a == 0) ? (G.fe[a][0] > 1 ? fidx : 0) : (G.g0 > 1 ? x.i : 0);
    const int xj = (a == 1) ? (G.fe[a][1] > 1 ? fidx : 0) : (G.g1 > 1 ? x.j : 0);
    const int xk = (a == 2) ? (G.fe[a][2] > 1 ? fidx : 0) : (G.g2 > 1 ? x.k : 0);
    return (xk * G.fe[a][1] + xj) * G.fe[a][0] + xi;
}

__device__ __forceinline__ int axis_coord(const Cell &x, int a) {
    return a == 0 ? x.i : (a == 1 ? x.j : x.k);
}
__device__ __forceinline__ int axis_len(const DevGrid &G, int a) {
    return a == 0 ? G.n0 : (a == 1 ? G.n1 : G.n2);
}
__device__ __forceinline__ long long axis_stride(const DevGrid &G, int a) {
    return a == 0 ? 1LL : (a == 1 ? (long long)G.n0 : (long long)G.n0 * G.n1);
}

// Intensity of direction n in the cell `o` steps along axis a from x, with
// boundary conditions applied: periodic wrap, or (outflow/vacuum) a copy of
// the adjacent active cell for directions leaving the domain through that
// boundary face and zero for directions entering it.
template <typename Real>
__device__ __forceinline__ Real nbr(const DevGrid &G, const Real *__restrict__ I, const Cell &x,
                                    int a, int o, int n) {
    const int coord = axis_coord(x, a);
    const int len = axis_len(G, a);
    const long long stride = axis_stride(G, a);
    const int idx = coord + o;
    if (idx >= 0 && idx < len) return I[(x.c + (long long)o * stride) * G.nang + n];
    const int side = idx < 0 ? 0 : 1;
    if (G.bc[a][side] == RT_BC_PERIODIC) {
        const int w = ((idx % len) + len) % len;
        return I[(x.c + (long long)(w - coord) * stride) * G.nang + n];
    }
    const int fg = face_geo(G, a, side ? len : 0, x);
    const int s = G.sgn[a][(size_t)fg * G.nang + n];
    const bool out = side ? (s > 0) : (s < 0);
    if (!out) return Real(0);
    const int edge = side ? len - 1 : 0;
    return I[(x.c + (long long)(edge - coord) * stride) * G.nang + n];
}

// div + w I as one rounding (every kernel's angular gather adds its edge
// terms this way, so they agree bit for bit)
template <typename Real>
__device__ __forceinline__ Real ang_fma(Real w, Real I, Real div) {
    if constexpr (sizeof(Real) == 4)
        return __builtin_fmaf(w, I, div);
    else
        return __builtin_fma(w, I, div);
}

// I* of direction n in cell x after the flux divergence (Sec. 2.2 gray
// integral form) and primitive recovery, zero where masked.  Adds the
// luminosity-face and masked-energy contributions to the accumulators.
template <typename Real>
__device__ __forceinline__ Real transport_dir(const DevGrid &G, const Real *__restrict__ Iin,
                                              const Cell &x, int n, Real dtR, Real ivol,
                                              double &lum_acc, double &me_acc) {
    const int N = G.nang;
    const Real *q = static_cast<const Real *>(G.q);
    const Real *vw = static_cast<const Real *>(G.vw);
    const Real Ic = Iin[x.c * N + n];
    Real dq = Real(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int coord = axis_coord(x, a);
        const int len = axis_len(G, a);
        Real v[5];
        v[2] = Ic;
        v[1] = nbr(G, Iin, x, a, -1, n);
        v[3] = nbr(G, Iin, x, a, +1, n);
        Real hlm = Real(0), hl0 = Real(0), hlp = Real(0);
        if (G.recon == RT_RECON_PLM) {
            v[0] = nbr(G, Iin, x, a, -2, n);
            v[4] = nbr(G, Iin, x, a, +2, n);
            hlm = half_slope(v[0], v[1], v[2]);
            hl0 = half_slope(v[1], v[2], v[3]);
            hlp = half_slope(v[2], v[3], v[4]);
        }
        const int flo = face_geo(G, a, coord, x);
        const int fhi = face_geo(G, a, coord + 1, x);
        const Real *C = static_cast<const Real *>(G.C[a]);
        const int slo = G.sgn[a][(size_t)flo * N + n];
        const int shi = G.sgn[a][(size_t)fhi * N + n];
        const Real ulo = slo > 0 ? v[1] + hlm : (slo < 0 ? v[2] - hl0 : Real(0));
        const Real uhi = shi > 0 ? v[2] + hl0 : (shi < 0 ? v[3] - hlp : Real(0));
        const Real Flo = C[(size_t)flo * N + n] * ulo;
        const Real Fhi = C[(size_t)fhi * N + n] * uhi;
        dq += Fhi - Flo;
        if (a == G.lum_axis) {
            if (G.lum_side == 1 && coord == len - 1) lum_acc -= G.domega[n] * (double)Fhi;
            if (G.lum_side == 0 && coord == 0) lum_acc += G.domega[n] * (double)Flo;
        }
    }
    Real div = Real(0);
    if (G.has_edges) {
#pragma unroll
        for (int s = 0; s < kMaxNbr; ++s) {
            const int e = G.adj_e[n * kMaxNbr + s];
            if (e < 0) break;
            const size_t vi = ((size_t)x.gc * G.nedge + e) * 2;
            const Real vv = vw[vi], ww = vw[vi + 1];
            const Real up = vv > Real(0) ? Iin[x.c * N + G.edge_lo[e]]
                                         : (vv < Real(0) ? Iin[x.c * N + G.edge_hi[e]] : Real(0));
            div = ang_fma(G.adj_s[n * kMaxNbr + s] > 0 ? ww : -ww, up, div);
        }
    }
    const Real qn = q[(size_t)x.gc * N + n];
    const Real Qs = qn * Ic - dtR * ivol * dq - quot(dtR * div, Real(G.domega[n]));
    if (G.mask[(size_t)x.gc * N + n]) {
        me_acc -= G.volD[x.gc] * G.domega[n] * (double)Qs;
        return Real(0);
    }
    return quot(Qs, qn);
}

// Row pointers of one axis for the general step: the cell is uniform across
// the wavefront, so its neighbour rows and face geometry rows are resolved
// once per cell and axis (boundary conditions included); each direction then
// loads row[n], one lane offset shared by all loads of a direction.
template <typename Real>
struct AxisRows {
    const Real *nb[4];            // rows at offsets -2, -1, +1, +2
    const int8_t *bs[4];          // outflow ghost: sign row of the boundary face, else nullptr
    const Real *Clo, *Chi;        // face coefficients of the lower/upper face
    const int8_t *Slo, *Shi;
    bool ghost;                   // some offset lands on an outflow/vacuum ghost
    bool lum_lo, lum_hi;          // lower/upper face is the luminosity face
    // optical-depth-aware flux: f of the lower/upper face and the fluid
    // (u^0^, u^a^) of the cells at offsets -1, 0, +1
    double f_lo, f_hi, u0n[3], un[3][3];
};

// Fluid data of the optical-depth-aware flux along axis a (Sec. 2, flux
// calculation): f = -expm1(-tau^2) of both faces of the cell, tau =
// tau_coeff alpha_E dt / u^0^ from the two adjacent cells' averages; a ghost
// neighbour carries the fluid of the cell it copies (outflow) or wraps to.
template <typename Real>
__device__ __forceinline__ void axis_fluid(const DevGrid &G, const Cell &x, int a,
                                           const double *__restrict__ rho,
                                           const double *__restrict__ uvec,
                                           const double *__restrict__ kap_a,
                                           const double *__restrict__ kap_s, double dt,
                                           AxisRows<Real> &R) {
    const int coord = axis_coord(x, a);
    const int len = axis_len(G, a);
    const long long stride = axis_stride(G, a);
    double aE[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int idx = coord + k - 1;
        if (idx < 0 || idx >= len) {
            const int side = idx < 0 ? 0 : 1;
            idx = G.bc[a][side] == RT_BC_PERIODIC ? ((idx % len) + len) % len : coord;
        }
        const long long c = x.c + (long long)(idx - coord) * stride;
        const double u1 = uvec[3 * c], u2 = uvec[3 * c + 1], u3 = uvec[3 * c + 2];
        R.un[k][0] = u1;
        R.un[k][1] = u2;
        R.un[k][2] = u3;
        R.u0n[k] = sqrt(1.0 + u1 * u1 + u2 * u2 + u3 * u3);
        aE[k] = (kap_a[c] + kap_s[c]) * rho[c];
    }
    const double tlo = G.tau_coeff * (0.5 * (aE[0] + aE[1])) * dt / (0.5 * (R.u0n[0] + R.u0n[1]));
    const double thi = G.tau_coeff * (0.5 * (aE[1] + aE[2])) * dt / (0.5 * (R.u0n[1] + R.u0n[2]));
    R.f_lo = -expm1(-tlo * tlo);
    R.f_hi = -expm1(-thi * thi);
}

// Flux factors (1 + (g - g_L), 1 + (g - g_R)) of a face with interpolating
// factor f between cells with fluid-frame n^0bar nL and nR (tau_face_inv:
// from 1/nL and 1/nR, formed once per cell where a cell borders two faces,
// by the refined hardware reciprocal in every kernel).
__device__ __forceinline__ void tau_face_inv(double f, double inL, double inR, double &facL,
                                             double &facR) {
    const double gL = -f * (1.0 + inL), gR = -f * (1.0 + inR);
    const double g = 0.5 * (gL + gR);
    facL = 1.0 + (g - gL);
    facR = 1.0 + (g - gR);
}
__device__ __forceinline__ void tau_face(double f, double nL, double nR, double &facL, double &facR) {
    tau_face_inv(f, rcp64(nL), rcp64(nR), facL, facR);
}

template <typename Real>
__device__ __forceinline__ void axis_rows(const DevGrid &G, const Real *__restrict__ Iin,
                                          const Cell &x, int a, AxisRows<Real> &R) {
    const int N = G.nang;
    const int coord = axis_coord(x, a);
    const int len = axis_len(G, a);
    const long long stride = axis_stride(G, a);
    R.ghost = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int o = k < 2 ? k - 2 : k - 1;
        const int idx = coord + o;
        R.bs[k] = nullptr;
        if (idx >= 0 && idx < len) {
            R.nb[k] = Iin + (x.c + (long long)o * stride) * N;
        } else {
            const int side = idx < 0 ? 0 : 1;
            if (G.bc[a][side] == RT_BC_PERIODIC) {
                const int w = ((idx % len) + len) % len;
                R.nb[k] = Iin + (x.c + (long long)(w - coord) * stride) * N;
            } else {
                const int edge = side ? len - 1 : 0;
                R.nb[k] = Iin + (x.c + (long long)(edge - coord) * stride) * N;
                R.bs[k] = G.sgn[a] + (size_t)face_geo(G, a, side ? len : 0, x) * N;
                R.ghost = true;
            }
        }
    }
    const int flo = face_geo(G, a, coord, x), fhi = face_geo(G, a, coord + 1, x);
    R.Clo = static_cast<const Real *>(G.C[a]) + (size_t)flo * N;
    R.Chi = static_cast<const Real *>(G.C[a]) + (size_t)fhi * N;
    R.Slo = G.sgn[a] + (size_t)flo * N;
    R.Shi = G.sgn[a] + (size_t)fhi * N;
    R.lum_lo = a == G.lum_axis && G.lum_side == 0 && coord == 0;
    R.lum_hi = a == G.lum_axis && G.lum_side == 1 && coord == len - 1;
}

// Contribution of one axis to the flux divergence of direction n (the same
// arithmetic as transport_dir, so the same I* bit for bit).  GHOST: some
// neighbour along this axis is an outflow/vacuum ghost.
template <bool GHOST, typename Real, bool TAU = false>
__device__ __forceinline__ Real axis_div(const DevGrid &G, const AxisRows<Real> &R, Real Ic, int n,
                                         double &lum_acc) {
    Real v[5];
    v[2] = Ic;
    const bool plm = G.recon == RT_RECON_PLM;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int slot = k < 2 ? k : k + 1;
        if ((k == 0 || k == 3) && !plm) {
            v[slot] = Real(0);
            continue;
        }
        Real val = R.nb[k][n];
        if constexpr (GHOST) {
            if (R.bs[k] != nullptr) {
                // ghost beyond a lower (k < 2) or upper face: the edge cell
                // for directions leaving through it, else zero
                const int s = R.bs[k][n];
                const bool out = k < 2 ? (s < 0) : (s > 0);
                val = out ? val : Real(0);
            }
        }
        v[slot] = val;
    }
    Real hlm = Real(0), hl0 = Real(0), hlp = Real(0);
    if (plm) {
        hlm = half_slope(v[0], v[1], v[2]);
        hl0 = half_slope(v[1], v[2], v[3]);
        hlp = half_slope(v[2], v[3], v[4]);
    }
    const int slo = R.Slo[n], shi = R.Shi[n];
    Real ulo = slo > 0 ? v[1] + hlm : (slo < 0 ? v[2] - hl0 : Real(0));
    Real uhi = shi > 0 ? v[2] + hl0 : (shi < 0 ? v[3] - hlp : Real(0));
    if constexpr (TAU) {
        double nb[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            nb[k] = R.u0n[k] - (R.un[k][0] * G.nhat[3 * n] + R.un[k][1] * G.nhat[3 * n + 1] +
                                R.un[k][2] * G.nhat[3 * n + 2]);
        double fL, fR;
        tau_face(R.f_lo, nb[0], nb[1], fL, fR);
        ulo *= Real(slo > 0 ? fL : fR);
        tau_face(R.f_hi, nb[1], nb[2], fL, fR);
        uhi *= Real(shi > 0 ? fL : fR);
    }
    const Real Flo = R.Clo[n] * ulo;
    const Real Fhi = R.Chi[n] * uhi;
    if (R.lum_hi) lum_acc -= G.domega[n] * (double)Fhi;
    if (R.lum_lo) lum_acc += G.domega[n] * (double)Flo;
    return Fhi - Flo;
}

// Largest direction count of the general kernels (8 chunks of 64 lanes).
constexpr int kMaxAngGeneral = 8 * kWave;

// Edge record of slot s of direction n (i = n * kMaxNbr + s): the edge index
// (bits 0-14), the direction across the edge (bits 15-29) and whether n is
// the edge's lo end (bit 30); -1 where the polygon has no such edge.
__device__ __forceinline__ int edge_record(const DevGrid &G, int i) {
    const int e = G.adj_e[i];
    if (e < 0) return -1;
    const bool is_lo = G.adj_s[i] > 0;
    const int m = is_lo ? G.edge_hi[e] : G.edge_lo[e];
    return e | (m << 15) | ((is_lo ? 1 : 0) << 30);
}

// Angular-flux divergence of direction n from staged edge records: with
// the edge's signed weight +-w (+ when n is the edge's lower direction) and
// the upwind direction's intensity, div = sum over the edges of +-w I_up.
template <typename Real>
__device__ __forceinline__ Real angular_div_rec(const int *__restrict__ rec, const Real *__restrict__ own,
                                                const Real *__restrict__ vwrow, int n) {
    Real div = Real(0);
    const Real In = own[n];
#pragma unroll
    for (int s = 0; s < kMaxNbr; ++s) {
        const int r = rec[n * kMaxNbr + s];
        if (r < 0) break;
        const int e = r & 0x7fff, m = (r >> 15) & 0x7fff;
        const bool is_lo = (r >> 30) & 1;
        const Real vv = vwrow[2 * e], ww = vwrow[2 * e + 1];
        const Real Im = own[m];
        const Real Ilo = is_lo ? In : Im, Ihi = is_lo ? Im : In;
        const Real up = vv > Real(0) ? Ilo : (vv < Real(0) ? Ihi : Real(0));
        div = ang_fma(is_lo ? ww : -ww, up, div);
    }
    return div;
}

// MAPR gradient of direction n (geodesic grids, Sec. 2.6), in the tangent
// coordinates of n: over the candidate planes through n and two consecutive
// neighbours, the one of smallest |g|; among planes within a relative
// tolerance of the smallest (ties that the grid's symmetry produces), the
// first in the neighbour order.  The tolerance sits well above the rounding
// of the intensity precision: 1e-10 in FP64, 1e-5 in FP32.
template <typename Real>
__device__ __forceinline__ Real mapr_tie() { return sizeof(Real) == 8 ? Real(1e-10) : Real(1e-5); }
// (Mn: direction n's candidate matrices, entry 4 i + j at Mn[(4 i + j) ms];
// nbn: its neighbours, slot s at nbn[s ns]; the general kernel reads the
// direction-major tables, the column kernel component-major copies in LDS)
template <typename Real>
__device__ __forceinline__ void mapr_gradient_t(int k, const int *__restrict__ nbn, int ns,
                                                const Real *__restrict__ Mn, int ms,
                                                const Real *__restrict__ own, int n, Real &gx,
                                                Real &gy) {
    const Real Ic = own[n];
    Real d[kMaxNbr];
#pragma unroll
    for (int s = 0; s < kMaxNbr; ++s) d[s] = own[nbn[s * ns]] - Ic;
    Real cx[kMaxNbr], cy[kMaxNbr], cq[kMaxNbr];
    Real qmin = Real(0);
#pragma unroll
    for (int i = 0; i < kMaxNbr; ++i) {
        const Real a = d[i], b = d[i + 1 < k ? i + 1 : 0];
        // every product-sum as written out fused multiply-adds, so every
        // kernel rounds the candidate slopes (and takes the ties) alike
        cx[i] = ang_fma(Mn[(4 * i + 1) * ms], b, Mn[(4 * i) * ms] * a);
        cy[i] = ang_fma(Mn[(4 * i + 3) * ms], b, Mn[(4 * i + 2) * ms] * a);
        cq[i] = ang_fma(cy[i], cy[i], cx[i] * cx[i]);
        if (i < k && (i == 0 || cq[i] < qmin)) qmin = cq[i];
    }
    const Real lim = qmin * (Real(1) + mapr_tie<Real>());
    gx = cx[0];
    gy = cy[0];
#pragma unroll
    for (int i = kMaxNbr - 1; i >= 0; --i)
        if (i < k && cq[i] <= lim) {
            gx = cx[i];
            gy = cy[i];
        }
}
template <typename Real>
__device__ __forceinline__ void mapr_gradient(const DevGrid &G, const Real *__restrict__ own, int n,
                                              Real &gx, Real &gy) {
    mapr_gradient_t(G.mapr_cnt[n], G.mapr_nb + n * kMaxNbr, 1,
                    static_cast<const Real *>(G.mapr_inv) + (size_t)n * kMaxNbr * 4, 1, own, n, gx,
                    gy);
}

// angular_div with MAPR face values: I + g . d at the edge midpoint, g of
// the cell the value is taken from (grad holds (gx, gy) per direction; Dm
// the edge midpoints' offsets, four per edge).
template <typename Real>
__device__ __forceinline__ Real angular_div_mapr_t(const Real *__restrict__ Dm,
                                                   const int *__restrict__ rec,
                                                   const Real *__restrict__ own,
                                                   const Real *__restrict__ vwrow,
                                                   const Real *grad, int n) {
    Real div = Real(0);
#pragma unroll
    for (int s = 0; s < kMaxNbr; ++s) {
        const int r = rec[n * kMaxNbr + s];
        if (r < 0) break;
        const int e = r & 0x7fff, m = (r >> 15) & 0x7fff;
        const bool is_lo = (r >> 30) & 1;
        const int lo = is_lo ? n : m, hi = is_lo ? m : n;
        const Real vv = vwrow[2 * e], ww = vwrow[2 * e + 1];
        const Real *D = Dm + 4 * e;
        const Real Ilo = ang_fma(grad[2 * lo + 1], D[1], ang_fma(grad[2 * lo], D[0], own[lo]));
        const Real Ihi = ang_fma(grad[2 * hi + 1], D[3], ang_fma(grad[2 * hi], D[2], own[hi]));
        const Real up = vv > Real(0) ? Ilo : (vv < Real(0) ? Ihi : Real(0));
        div = ang_fma(is_lo ? ww : -ww, up, div);
    }
    return div;
}
template <typename Real>
__device__ __forceinline__ Real angular_div_mapr(const DevGrid &G, const int *__restrict__ rec,
                                                 const Real *__restrict__ own,
                                                 const Real *__restrict__ vwrow,
                                                 const Real *grad, int n) {
    return angular_div_mapr_t(static_cast<const Real *>(G.mapr_d), rec, own, vwrow, grad, n);
}

// angular_div with PLM face values (latitude-longitude grids, Sec. 2.3):
// the lo side's value I_lo + delta/2 from (I_ll, I_lo, I_hi) and the hi
// side's I_hi - delta/2 from (I_lo, I_hi, I_rr); both cells of an edge form
// the same expression, so the fluxes telescope exactly.
// (ell, err: each edge's outer stencil directions, from the device tables or
// an LDS copy)
template <typename Real>
__device__ __forceinline__ Real angular_div_plm_t(const int *__restrict__ ell,
                                                  const int *__restrict__ err,
                                                  const int *__restrict__ rec,
                                                  const Real *__restrict__ own,
                                                  const Real *__restrict__ vwrow, int n) {
    Real div = Real(0);
    const Real In = own[n];
#pragma unroll
    for (int s = 0; s < kMaxNbr; ++s) {
        const int r = rec[n * kMaxNbr + s];
        if (r < 0) break;
        const int e = r & 0x7fff, m = (r >> 15) & 0x7fff;
        const bool is_lo = (r >> 30) & 1;
        const Real vv = vwrow[2 * e], ww = vwrow[2 * e + 1];
        const Real Im = own[m];
        const Real Ilo = is_lo ? In : Im, Ihi = is_lo ? Im : In;
        const Real IL = Ilo + half_slope(own[ell[e]], Ilo, Ihi);
        const Real IR = Ihi - half_slope(Ilo, Ihi, own[err[e]]);
        const Real up = vv > Real(0) ? IL : (vv < Real(0) ? IR : Real(0));
        div = ang_fma(is_lo ? ww : -ww, up, div);
    }
    return div;
}
template <typename Real>
__device__ __forceinline__ Real angular_div_plm(const DevGrid &G, const int *__restrict__ rec,
                                                const Real *__restrict__ own,
                                                const Real *__restrict__ vwrow, int n) {
    return angular_div_plm_t(G.edge_ll, G.edge_rr, rec, own, vwrow, n);
}

}  // namespace rt
