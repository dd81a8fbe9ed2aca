// Adjoint of the transport for spatially uniform geometry, tiled like the
// forward fast path (Sec. 2.3-2.4 reversed).
//
// In the coordinate t that increases along the direction's motion on an
// axis, the face between cells t-1 and t carries the upwind PLM value
//   V_t = I_{t-1} + h(I_{t-2}, I_{t-1}, I_t),  h(l,m,r) = (m-l)(r-m)/(r-l)
// (half the van Leer slope, 0 unless the two differences share a sign), and
// the flux divergence of cell x is c (V_{x+1} - V_x) with the signed
// coefficient c = sgn C / dV.  With psi = dJ/dQ* (Q* = n^0 n_0 I*), the face
// adjoint is L_t = dt c (psi_t - psi_{t-1}) plus, on the luminosity face, the
// seed of J, and
//   dJ/dI_x = q psi_x + sum_axes [ L_x  dh(I_{x-2},I_{x-1},I_x)/dr
//                                 + L_{x+1} (1 + dh(I_{x-1},I_x,I_{x+1})/dm)
//                                 + L_{x+2} dh(I_x,I_{x+1},I_{x+2})/dl ],
// with dh/dl = -b^2/s^2, dh/dm = (b^2 - a^2)/s^2, dh/dr = a^2/s^2 for
// a = m - l, b = r - m, s = a + b, evaluated on the branch (a b > 0 or not)
// that the forward step took: the product is formed from the same two
// differences, so the branch decision is bitwise the same.
//
// Work decomposition: a workgroup owns a 4x4 tile of cells and a chunk of
// NC * SW directions (the transport adjoint has no sums over directions, so
// the direction range splits freely) and marches along axis 2.  Axis-0/1
// neighbours of I and psi come from LDS planes with a two-cell cross halo;
// along axis 2 each face is evaluated once, when the march first reaches a
// plane that needs it, and its three contributions (to the planes z, z+1,
// z+2) are carried forward in registers.
#include <hip/hip_runtime.h>

#include "k_common.h"
#include "k_tile.h"

namespace rt {
namespace {

// Derivatives of h(l, m, r) with respect to one of its arguments.
template <typename Real>
__device__ __forceinline__ Real inv(Real s) {
    if constexpr (sizeof(Real) == 4)
        return __builtin_amdgcn_rcpf(s);
    else
        return rcp64(s);
}
template <typename Real>
__device__ __forceinline__ Real dh_dr(Real l, Real m, Real r) {
    const Real a = m - l, b = r - m;
    if (!(a * b > Real(0))) return Real(0);
    const Real x = a * inv(a + b);
    return x * x;
}
template <typename Real>
__device__ __forceinline__ Real dh_dm(Real l, Real m, Real r) {
    const Real a = m - l, b = r - m;
    if (!(a * b > Real(0))) return Real(0);
    const Real i = inv(a + b);
    const Real x = a * i, y = b * i;
    return y * y - x * x;
}
template <typename Real>
__device__ __forceinline__ Real dh_dl(Real l, Real m, Real r) {
    const Real a = m - l, b = r - m;
    if (!(a * b > Real(0))) return Real(0);
    const Real y = b * inv(a + b);
    return -(y * y);
}

// the luminosity face along an axis of length len: face index F lies on it
__device__ __forceinline__ bool lum_face(int F, int len, bool periodic, int side) {
    if (periodic) return F == 0 || F == len;
    return F == (side ? len : 0);
}

template <typename Real, int SW, int NC>
__global__ __launch_bounds__(kTC * SW) void k_adj_march(DevGrid G, MarchInfo M, int nchunk, int P,
                                                        const Real *__restrict__ Iin,
                                                        const Real *__restrict__ psi, double dt,
                                                        double lum_weight,
                                                        Real *__restrict__ lam) {
    constexpr int NT = kTC * SW;
    constexpr int NP = NC * SW;   // directions per chunk
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_hrow[kHalo];
    __shared__ unsigned s_htest[kHalo];

    const int N = G.nang;
    const int per = gridDim.x / 8;
    const int logical = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (logical >= M.nwork * nchunk) return;
    const int chunk = logical % nchunk;
    const int work = logical / nchunk;
    const int d0 = chunk * NP;
    Seg sg;
    {
        const int tile = work / M.nseg, seg = work % M.nseg;
        sg.tx0 = (tile % M.ntx) * kTX;
        sg.ty0 = (tile / M.ntx) * kTY;
        sg.z0 = seg * M.seglen;
        sg.z1 = min(G.n2, sg.z0 + M.seglen);
    }

    // LDS: per-direction tables of the chunk (neutral values past N), then
    // the current plane of I and of psi (tile + halo)
    Real *s_q = reinterpret_cast<Real *>(smem);   // [NP] q
    Real *s_c = s_q + NP;                         // [3][NP] dt * signed coefficient
    Real *s_lw = s_c + 3 * NP;                    // [NP] luminosity-face seed
    Real *s_I = s_lw + NP;                        // [kPlane][P]
    Real *s_P = s_I + kPlane * P;                 // [kPlane][P]
    unsigned char *s_bits = reinterpret_cast<unsigned char *>(s_P + kPlane * P);   // [NP]

    const int la = G.lum_axis, lside = G.lum_side;
    for (int i = threadIdx.x; i < NP; i += NT) {
        const int n = d0 + i;
        const bool live = n < N;
        const int j = live ? n : 0;
        const unsigned b = live ? M.bits[j] : 0u;
        const double c[3] = {(double)static_cast<const Real *>(M.cx)[j],
                             (double)static_cast<const Real *>(M.cy)[j],
                             (double)static_cast<const Real *>(M.cz)[j]};
        s_q[i] = live ? static_cast<const Real *>(M.q)[j] : Real(0);
        for (int ax = 0; ax < 3; ++ax) s_c[ax * NP + i] = live ? Real(dt * c[ax]) : Real(0);
        // dJ/dV on the luminosity face: J gains -w dt dOmega dV F, F = +c V
        // when the motion leaves through the face, -c V when it enters
        const bool neg = (b & (2u << (2 * la))) != 0;
        const double outward = (neg == (lside == 0)) ? 1.0 : -1.0;
        s_lw[i] = live ? Real(-lum_weight * dt * G.domega[j] * M.vol * c[la] * outward) : Real(0);
        s_bits[i] = (unsigned char)b;
    }
    if (threadIdx.x < kHalo) {
        const int h = threadIdx.x;
        int x, y;
        halo_pos(h, x, y);
        int gx = sg.tx0 + x, gy = sg.ty0 + y;
        unsigned test = 0;
        if (gx < 0 || gx >= G.n0) {
            const int side = gx < 0 ? 0 : 1;
            if (G.bc[0][side] == RT_BC_PERIODIC) {
                gx = ((gx % G.n0) + G.n0) % G.n0;
            } else {
                test = side ? kXP : kXN;
                gx = side ? G.n0 - 1 : 0;
            }
        }
        if (gy < 0 || gy >= G.n1) {
            const int side = gy < 0 ? 0 : 1;
            if (G.bc[1][side] == RT_BC_PERIODIC) {
                gy = ((gy % G.n1) + G.n1) % G.n1;
            } else {
                test = side ? kYP : kYN;
                gy = side ? G.n1 - 1 : 0;
            }
        }
        s_hrow[h] = (long long)gy * G.n0 + gx;
        s_htest[h] = test;
    }
    __syncthreads();

    const int lane = threadIdx.x % kWave;
    const int a = lane % SW;
    const int cl = threadIdx.x / SW;
    const int tx = cl % kTX, ty = cl / kTX;
    const int gx = sg.tx0 + tx, gy = sg.ty0 + ty;
    const long long pcells = (long long)G.n0 * G.n1;
    const long long row = (long long)gy * G.n0 + gx;
    const bool plm = G.recon == RT_RECON_PLM;
    const int o_c = plane_slot(tx, ty) * P;
    const int ox[4] = {plane_slot(tx - 2, ty) * P, plane_slot(tx - 1, ty) * P,
                       plane_slot(tx + 1, ty) * P, plane_slot(tx + 2, ty) * P};
    const int oy[4] = {plane_slot(tx, ty - 2) * P, plane_slot(tx, ty - 1) * P,
                       plane_slot(tx, ty + 1) * P, plane_slot(tx, ty + 2) * P};
    const bool zper = G.bc[2][0] == RT_BC_PERIODIC;
    // faces gx-1 .. gx+2 (or gy-1 .. gy+2) of this cell on the luminosity face
    unsigned lmask = 0;
    if (la < 2) {
        const int c0 = la == 0 ? gx : gy;
        const int len = la == 0 ? G.n0 : G.n1;
        const bool per_ax = G.bc[la][0] == RT_BC_PERIODIC;
        for (int j = 0; j < 4; ++j)
            if (lum_face(c0 - 1 + j, len, per_ax, lside)) lmask |= 1u << j;
    }
    const bool lum_xy = __ballot(lmask != 0) != 0;   // wave-uniform

    // intensities of plane pz of a row with the boundary conditions applied
    // (as in the forward step); psi is zero outside a non-periodic boundary
    auto load_I = [&](int pz, long long r, unsigned xytest, Real *dst) {
        long long zz = pz;
        unsigned test = xytest;
        if (pz < 0 || pz >= G.n2) {
            const int side = pz < 0 ? 0 : 1;
            if (G.bc[2][side] == RT_BC_PERIODIC) {
                zz = ((pz % G.n2) + G.n2) % G.n2;
            } else {
                test |= side ? kZP : kZN;
                zz = side ? G.n2 - 1 : 0;
            }
        }
        const Real *src = Iin + (zz * pcells + r) * N;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int i = a + SW * k;
            const Real v = src[min(d0 + i, N - 1)];
            dst[k] = ((s_bits[i] & test) == test) ? v : Real(0);
        }
    };
    auto load_P = [&](int pz, long long r, bool inside, Real *dst) {
        long long zz = pz;
        if (pz < 0 || pz >= G.n2) {
            if (zper) {
                zz = ((pz % G.n2) + G.n2) % G.n2;
            } else {
                inside = false;
                zz = 0;
            }
        }
        const Real *src = psi + (zz * pcells + r) * N;
#pragma unroll
        for (int k = 0; k < NC; ++k) dst[k] = inside ? src[min(d0 + a + SW * k, N - 1)] : Real(0);
    };
    long long hrow[kHPG];
    unsigned htest[kHPG];
#pragma unroll
    for (int j = 0; j < kHPG; ++j) {
        hrow[j] = s_hrow[kHPG * cl + j];
        htest[j] = s_htest[kHPG * cl + j];
    }

    // Axis-2 face whose upwind stencil is planes (p, p+1, p+2): the face
    // between p+1 and p+2 for motion along +axis 2 (upwind cell p+1), between
    // p and p+1 for motion along -axis 2 (upwind cell p+1).  Its adjoint
    // times dV/dI goes to planes p, p+1, p+2 (tA, tB, tC).
    auto zface = [&](int p, const Real *A, const Real *B, const Real *Cc, const Real *PA,
                     const Real *PB, const Real *PC, Real *tA, Real *tB, Real *tC) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int i = a + SW * k;
            const bool nz = (s_bits[i] & kZN) != 0;
            Real L = s_c[2 * NP + i] * ((nz ? PA[k] : PC[k]) - PB[k]);
            if (la == 2) {
                const int F = nz ? p + 1 : p + 2;
                L += lum_face(F, G.n2, zper, lside) ? s_lw[i] : Real(0);
            }
            // V = B + sigma h(A, B, C), sigma = -1 for motion along -axis 2
            Real hA = Real(0), hB = Real(0), hC = Real(0);
            if (plm) {
                const Real da = B[k] - A[k], db = Cc[k] - B[k];
                if (da * db > Real(0)) {
                    const Real iv = inv(da + db);
                    const Real x = da * iv, y = db * iv;
                    hA = -(y * y);
                    hB = y * y - x * x;
                    hC = x * x;
                }
            }
            const Real Ls = nz ? -L : L;
            tA[k] = Ls * hA;
            tB[k] = L + Ls * hB;
            tC[k] = Ls * hC;
        }
    };

    // prologue: the two faces below the segment's first plane seed the carries
    Real Z0[NC], Z1[NC], Z2[NC], P0[NC], P1[NC], P2[NC], c1[NC], c2[NC];
    {
        Real tA[NC], tB[NC], tC[NC];
        load_I(sg.z0 - 2, row, 0u, Z0);
        load_I(sg.z0 - 1, row, 0u, Z1);
        load_I(sg.z0, row, 0u, Z2);
        load_P(sg.z0 - 2, row, true, P0);
        load_P(sg.z0 - 1, row, true, P1);
        load_P(sg.z0, row, true, P2);
        zface(sg.z0 - 2, Z0, Z1, Z2, P0, P1, P2, tA, tB, tC);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            c1[k] = tC[k];
            Z0[k] = Z1[k];
            Z1[k] = Z2[k];
            P0[k] = P1[k];
            P1[k] = P2[k];
        }
        load_I(sg.z0 + 1, row, 0u, Z2);
        load_P(sg.z0 + 1, row, true, P2);
        zface(sg.z0 - 1, Z0, Z1, Z2, P0, P1, P2, tA, tB, tC);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            c1[k] = c1[k] + tB[k];
            c2[k] = tC[k];
            Z0[k] = Z1[k];
            Z1[k] = Z2[k];
            P0[k] = P1[k];
            P1[k] = P2[k];
        }
        load_I(sg.z0 + 2, row, 0u, Z2);
        load_P(sg.z0 + 2, row, true, P2);
        // first plane into LDS
        Real h0[kHPG][NC], q0[kHPG][NC];
#pragma unroll
        for (int j = 0; j < kHPG; ++j) {
            load_I(sg.z0, hrow[j], htest[j], h0[j]);
            load_P(sg.z0, hrow[j], htest[j] == 0u, q0[j]);
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int i = a + SW * k;
            s_I[o_c + i] = Z0[k];
            s_P[o_c + i] = P0[k];
#pragma unroll
            for (int j = 0; j < kHPG; ++j) {
                s_I[(kTC + kHPG * cl + j) * P + i] = h0[j][k];
                s_P[(kTC + kHPG * cl + j) * P + i] = q0[j][k];
            }
        }
    }

    for (int z = sg.z0; z < sg.z1; ++z) {
        __syncthreads();
        const bool more = z + 1 < sg.z1;
        Real Zn[NC], Pn[NC], hI[kHPG][NC], hP[kHPG][NC];
        if (more) {
            load_I(z + 3, row, 0u, Zn);
            load_P(z + 3, row, true, Pn);
#pragma unroll
            for (int j = 0; j < kHPG; ++j) {
                load_I(z + 1, hrow[j], htest[j], hI[j]);
                load_P(z + 1, hrow[j], htest[j] == 0u, hP[j]);
            }
        }
        Real tA[NC], tB[NC], tC[NC];
        zface(z, Z0, Z1, Z2, P0, P1, P2, tA, tB, tC);
        Real *dst = lam + ((long long)z * pcells + row) * N;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int i = a + SW * k;
            const unsigned bits = s_bits[i];
            const bool nx = (bits & kXN) != 0, ny = (bits & kYN) != 0;
            Real out = s_q[i] * P0[k];
            // axis 0, neighbours in upwind order u-2 .. u+2 and psi p-1 .. p+2
            {
                const Real m2 = s_I[ox[0] + i], m1 = s_I[ox[1] + i];
                const Real p1 = s_I[ox[2] + i], p2 = s_I[ox[3] + i];
                const Real um2 = nx ? p2 : m2, um1 = nx ? p1 : m1;
                const Real up1 = nx ? m1 : p1, up2 = nx ? m2 : p2;
                const Real r2 = s_P[ox[0] + i], r1 = s_P[ox[1] + i];
                const Real s1 = s_P[ox[2] + i], s2 = s_P[ox[3] + i];
                const Real qm1 = nx ? s1 : r1, qp1 = nx ? r1 : s1, qp2 = nx ? r2 : s2;
                const Real c = s_c[i];
                Real L0 = c * (P0[k] - qm1), L1 = c * (qp1 - P0[k]), L2 = c * (qp2 - qp1);
                if (la == 0 && lum_xy) {
                    const Real w = s_lw[i];
                    L0 += (lmask >> (nx ? 2 : 1)) & 1u ? w : Real(0);
                    L1 += (lmask >> (nx ? 1 : 2)) & 1u ? w : Real(0);
                    L2 += (lmask >> (nx ? 0 : 3)) & 1u ? w : Real(0);
                }
                if (plm)
                    out += L0 * dh_dr(um2, um1, Z0[k]) + L1 * (Real(1) + dh_dm(um1, Z0[k], up1)) +
                           L2 * dh_dl(Z0[k], up1, up2);
                else
                    out += L1;
            }
            // axis 1
            {
                const Real m2 = s_I[oy[0] + i], m1 = s_I[oy[1] + i];
                const Real p1 = s_I[oy[2] + i], p2 = s_I[oy[3] + i];
                const Real um2 = ny ? p2 : m2, um1 = ny ? p1 : m1;
                const Real up1 = ny ? m1 : p1, up2 = ny ? m2 : p2;
                const Real r2 = s_P[oy[0] + i], r1 = s_P[oy[1] + i];
                const Real s1 = s_P[oy[2] + i], s2 = s_P[oy[3] + i];
                const Real qm1 = ny ? s1 : r1, qp1 = ny ? r1 : s1, qp2 = ny ? r2 : s2;
                const Real c = s_c[NP + i];
                Real L0 = c * (P0[k] - qm1), L1 = c * (qp1 - P0[k]), L2 = c * (qp2 - qp1);
                if (la == 1 && lum_xy) {
                    const Real w = s_lw[i];
                    L0 += (lmask >> (ny ? 2 : 1)) & 1u ? w : Real(0);
                    L1 += (lmask >> (ny ? 1 : 2)) & 1u ? w : Real(0);
                    L2 += (lmask >> (ny ? 0 : 3)) & 1u ? w : Real(0);
                }
                if (plm)
                    out += L0 * dh_dr(um2, um1, Z0[k]) + L1 * (Real(1) + dh_dm(um1, Z0[k], up1)) +
                           L2 * dh_dl(Z0[k], up1, up2);
                else
                    out += L1;
            }
            // axis 2: this plane's share of the new face plus the carries
            out += tA[k] + c1[k];
            c1[k] = c2[k] + tB[k];
            c2[k] = tC[k];
            if (d0 + i < N) dst[d0 + i] = out;
        }
        __syncthreads();
        if (more) {
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int i = a + SW * k;
                s_I[o_c + i] = Z1[k];
                s_P[o_c + i] = P1[k];
#pragma unroll
                for (int j = 0; j < kHPG; ++j) {
                    s_I[(kTC + kHPG * cl + j) * P + i] = hI[j][k];
                    s_P[(kTC + kHPG * cl + j) * P + i] = hP[j][k];
                }
                Z0[k] = Z1[k];
                Z1[k] = Z2[k];
                Z2[k] = Zn[k];
                P0[k] = P1[k];
                P1[k] = P2[k];
                P2[k] = Pn[k];
            }
        }
    }
}

template <typename Real, int SW, int NC>
int launch_one(rt_grid *g, hipStream_t s, const Real *Iin, const Real *psi, double dt,
               double lum_weight, Real *lam) {
    const MarchInfo &M = g->march;
    const int NP = SW * NC;
    const int nchunk = (g->dg.nang + NP - 1) / NP;
    const int P = march_pstride(g->precision, NP);
    const size_t lds = (size_t)NP * (6 * sizeof(Real) + 1) + 2 * (size_t)kPlane * P * sizeof(Real);
    if (lds > 150 * 1024) return RT_EINVAL;
    if (ensure_dynamic_lds(reinterpret_cast<const void *>(&k_adj_march<Real, SW, NC>), lds) != RT_OK)
        return RT_EDEVICE;
    const long long total = (long long)M.nwork * nchunk;
    if (total >= (1LL << 30)) return RT_EINVAL;
    const int grid = (int)((total + 7) / 8 * 8);
    hipLaunchKernelGGL((k_adj_march<Real, SW, NC>), dim3(grid), dim3(kTC * SW), lds, s, g->dg, M,
                       nchunk, P, Iin, psi, dt, lum_weight, lam);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

}  // namespace

int launch_adj_march(rt_grid *g, hipStream_t s, const void *Iin, const void *psi, double dt,
                     double lum_weight, void *lam) {
    if (g->precision == RT_F32)
        return launch_one<float, 32, 3>(g, s, static_cast<const float *>(Iin),
                                        static_cast<const float *>(psi), dt, lum_weight,
                                        static_cast<float *>(lam));
    return launch_one<double, 32, 3>(g, s, static_cast<const double *>(Iin),
                                     static_cast<const double *>(psi), dt, lum_weight,
                                     static_cast<double *>(lam));
}

}  // namespace rt
