// Fused radiation step, fast path for geometry that is uniform in space (every
// geometry table depends on the direction only, no angular fluxes): e.g. flat
// spacetime in Cartesian coordinates with a constant tetrad (Sec. 2.2).
//
// Work decomposition (gfx950):
//   * a workgroup owns a 4x4 tile of cells in the (axis 0, axis 1) plane and
//     marches along axis 2 over a segment of planes;
//   * each cell of the tile is owned by a group of SW lanes (SW = 16 or
//     32); lane a of the group handles directions a, a+SW, ... (NC of them),
//     so the coupling's per-cell FP64 angle sums are SW-lane shuffles and the
//     quartic runs once per lane group, several cells per wavefront;
//   * axis-2 neighbours come from a five-plane register queue (each plane is
//     read from HBM once per segment), axis-0/1 neighbours from an LDS copy of
//     the current plane with a two-cell cross-shaped halo;
//   * PLM is evaluated on the upwind side only (a face needs only I_L or I_R);
//     each face value is computed by the same expression from the same inputs
//     in both cells that share it, so face fluxes telescope exactly; along
//     axis 2 the upper face value of a plane is kept for the next plane;
//   * workgroups are dispatched round-robin over the 8 XCDs; the logical tile
//     order is remapped so that each XCD owns a contiguous band of tiles and
//     halo rows hit its own L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "k_common.h"
#include "k_tile.h"

namespace rt {
namespace {

#ifndef RT_MARCH_WAVES_PER_EU
#define RT_MARCH_WAVES_PER_EU 2
#endif

// One stage of the two-stage integrator (STG = true): Q* = q (gI I + gB Ib)
// - beta dt (flux terms), the coupling starts from gT T + gTb Tb and runs over
// beta dt, and the bookkeeping and masked-energy ledger carry the weight wS.
template <typename Real>
struct MStage {
    const Real *Ib;
    const double *Tb;
    double gI, gB, beta, gT, gTb, wS;
};

template <typename Real, int SW, int NC, bool STG = false>
__global__ __launch_bounds__(kTC * SW) __attribute__((amdgpu_waves_per_eu(RT_MARCH_WAVES_PER_EU)))
void k_march(
    DevGrid G, MarchInfo M, const Real *__restrict__ Iin, Real *__restrict__ Iout,
    double *__restrict__ T, const double *__restrict__ rho, const double *__restrict__ uvec,
    const double *__restrict__ kap_a, const double *__restrict__ kap_s, double dt_step,
    double *__restrict__ dT0, double *__restrict__ partials, int *__restrict__ nr_partial,
    Real *__restrict__ Istar, MStage<Real> st) {
    const double dt = STG ? st.beta * dt_step : dt_step;   // this stage's time step
    constexpr int NT = kTC * SW;
    constexpr int NW = NT / kWave;
    constexpr int NP = NC * SW;               // padded direction count
    // FP32 planes are double-buffered (plane z+1 is written while plane z is
    // read, one barrier per plane); FP64 planes do not fit twice in LDS
    constexpr int NBUF = sizeof(Real) == 4 ? 2 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sh_l[NW], sh_m[NW];
    __shared__ int sh_n[NW];
    __shared__ long long s_hrow[kHalo];
    __shared__ unsigned s_htest[kHalo];
    __shared__ double s_fl[kTC][8];           // fluid state of the tile's cells
    __shared__ int s_beam[kTC];               // beam flag of the tile's cells
    __shared__ double s_E0[16];               // E0 of the (uniform) geometry

    const int N = G.nang;
    // XCD-aware remap: the hardware hands block b to XCD b % 8
    const int per = gridDim.x / 8;
    const int logical = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (logical >= M.nwork) {
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = 0.0;
            partials[2 * blockIdx.x + 1] = 0.0;
            nr_partial[blockIdx.x] = 0;
        }
        return;
    }
    Seg sg;
    {
        const int tile = logical / M.nseg, seg = logical % M.nseg;
        sg.tx0 = (tile % M.ntx) * kTX;
        sg.ty0 = (tile / M.ntx) * kTY;
        sg.z0 = seg * M.seglen;
        sg.z1 = min(G.n2, sg.z0 + M.seglen);
    }

    // LDS: per-direction tables padded to NP entries with neutral values,
    // then the current plane (tile + halo)
    double *s_nh = reinterpret_cast<double *>(smem);          // [3][NP]
    double *s_dom = s_nh + 3 * NP;                            // [NP] dOmega (0 if masked/pad)
    double *s_dom_all = s_dom + NP;                           // [NP] dOmega (0 if pad)
    Real *s_tab = reinterpret_cast<Real *>(s_dom_all + NP);   // [5][NP] q, 1/q, cx, cy, cz (signed)
    Real *s_pl = s_tab + 5 * NP;                              // [NBUF][kPlane][P]
    unsigned char *s_bits =
        reinterpret_cast<unsigned char *>(s_pl + NBUF * kPlane * M.pstride);   // [NP]
    const int P = M.pstride;

    for (int i = threadIdx.x; i < NP; i += NT) {
        const bool live = i < N;
        const int j = live ? i : 0;
        const unsigned b = live ? M.bits[j] : 0u;
        const bool masked = (b & kMasked) != 0;
        s_nh[i] = live ? G.nhat[3 * j] : 0.0;
        s_nh[NP + i] = live ? G.nhat[3 * j + 1] : 0.0;
        s_nh[2 * NP + i] = live ? G.nhat[3 * j + 2] : 0.0;
        s_dom_all[i] = live ? G.domega[j] : 0.0;
        s_dom[i] = (live && !masked) ? G.domega[j] : 0.0;
        s_tab[i] = live ? static_cast<const Real *>(M.q)[j] : Real(1);
        s_tab[NP + i] = live ? static_cast<const Real *>(M.iq)[j] : Real(1);
        s_tab[2 * NP + i] = live ? static_cast<const Real *>(M.cx)[j] : Real(0);
        s_tab[3 * NP + i] = live ? static_cast<const Real *>(M.cy)[j] : Real(0);
        s_tab[4 * NP + i] = live ? static_cast<const Real *>(M.cz)[j] : Real(0);
        s_bits[i] = (unsigned char)b;
    }
    // halo sources: row index inside a plane, and the flag bit a direction
    // must carry for an outflow/vacuum ghost to copy the edge cell
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
    if (threadIdx.x < 16) s_E0[threadIdx.x] = G.E0[threadIdx.x];
    __syncthreads();

    const int lane = threadIdx.x % kWave;
    const int a = lane % SW;
    const int cl = threadIdx.x / SW;            // tile cell owned by this lane group
    const int tx = cl % kTX, ty = cl / kTX;
    const int gx = sg.tx0 + tx, gy = sg.ty0 + ty;
    const long long pcells = (long long)G.n0 * G.n1;
    const long long row = (long long)gy * G.n0 + gx;
    const Real dtR = Real(dt);
    const bool plm = G.recon == RT_RECON_PLM;
    const double vol = M.vol;
    const double n0u = G.n0u[0];
    const double *E0 = s_E0;
    // LDS element offsets of this cell and its axis-0/1 neighbours (-2,-1,+1,+2)
    const int o_c = plane_slot(tx, ty) * P;
    const int ox[4] = {plane_slot(tx - 2, ty) * P, plane_slot(tx - 1, ty) * P,
                       plane_slot(tx + 1, ty) * P, plane_slot(tx + 2, ty) * P};
    const int oy[4] = {plane_slot(tx, ty - 2) * P, plane_slot(tx, ty - 1) * P,
                       plane_slot(tx, ty + 1) * P, plane_slot(tx, ty + 2) * P};
    // luminosity face weights of this cell (0 unless it touches the face)
    const int lside = G.lum_side;
    const bool on_lum_xy = (G.lum_axis == 0 && gx == (lside ? G.n0 - 1 : 0)) ||
                           (G.lum_axis == 1 && gy == (lside ? G.n1 - 1 : 0));

    // plane pz of a row, with the axis-2 boundary condition; `xytest` is the
    // axis-0/1 outflow test of a halo row (0: always copy)
    auto load_row = [&](int pz, long long r, unsigned xytest, Real *dst) {
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
            const int n = a + SW * k;
            dst[k] = src[k < NC - 1 ? n : min(n, N - 1)];
        }
        if (test != 0) {
            // ghost of an outflow/vacuum boundary: copy for directions leaving
            // through it (all bits of `test` set), zero for the others
#pragma unroll
            for (int k = 0; k < NC; ++k)
                dst[k] = ((s_bits[a + SW * k] & test) == test) ? dst[k] : Real(0);
        }
    };
    // this lane group's halo cells: source rows and outflow tests
    long long hrow[kHPG];
    unsigned htest[kHPG];
#pragma unroll
    for (int j = 0; j < kHPG; ++j) {
        hrow[j] = s_hrow[kHPG * cl + j];
        htest[j] = s_htest[kHPG * cl + j];
    }
    // one fluid field per lane (a < 7): u1 u2 u3 rho kappa_a kappa_s T.  With
    // FP32 intensities the lane's field address and stride are fixed here, so
    // the plane loop keeps one address per lane instead of five scalar
    // pointers (the scalar file is full); the FP64 kernel, at its VGPR limit,
    // keeps the pointers and selects per plane.
    const int fsel = a < 7 ? a : 6;
    const double *fbase = fsel < 3 ? uvec + fsel
                                   : (fsel == 3 ? rho : (fsel == 4 ? kap_a : (fsel == 5 ? kap_s : T)));
    const long long fstride = fsel < 3 ? 3 : 1;
    auto load_fluid = [&](int z) -> double {
        const long long c = (long long)z * pcells + row;
        if constexpr (sizeof(Real) == 4) {
            return fbase[fstride * c];
        } else {
            return fsel < 3 ? uvec[3 * c + fsel]
                            : (fsel == 3 ? rho[c] : (fsel == 4 ? kap_a[c] : (fsel == 5 ? kap_s[c] : T[c])));
        }
    };
    // the cell's beam flag, prefetched one plane ahead with the fluid state
    // (so the plane loop does not wait on a late load behind the next
    // plane's prefetch) and kept as loaded until lane 7 stores it
    auto load_beam = [&](int z) -> int {
        return G.beam != nullptr ? (int)G.beam[(long long)z * pcells + row] : 0;
    };

    // first plane of the segment into LDS: own cell from the queue, two halo
    // cells per lane group; later planes are written at the end of a step
    Real qz[5][NC];
#pragma unroll
    for (int p = 0; p < 5; ++p) load_row(sg.z0 - 2 + p, row, 0u, qz[p]);
    {
        Real h0[kHPG][NC];
#pragma unroll
        for (int j = 0; j < kHPG; ++j) load_row(sg.z0, hrow[j], htest[j], h0[j]);
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int n = a + SW * k;
            s_pl[o_c + n] = qz[2][k];
#pragma unroll
            for (int j = 0; j < kHPG; ++j) s_pl[(kTC + kHPG * cl + j) * P + n] = h0[j][k];
        }
        const double flv = load_fluid(sg.z0);
        if (a < 7) s_fl[cl][a] = flv;
        if (a == 7) s_beam[cl] = load_beam(sg.z0);
    }
    // Axis-2 face value carried from plane to plane.  The upper face of plane
    // z is the lower face of plane z+1, and both cells form its value with
    // the same expression from the same inputs, so it is formed once; the
    // lower face of the segment's first plane is formed here from the queue.
    Real zc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const bool nz = (s_bits[a + SW * k] & kZN) != 0;
        const Real l = nz ? qz[3][k] : qz[0][k];
        const Real m = nz ? qz[2][k] : qz[1][k];
        const Real r = nz ? qz[1][k] : qz[2][k];
        zc[k] = plm ? m + half_slope(l, m, r) : m;
    }

    // per-lane direction flags (loop invariant): motion along -axis 0/1/2, masked
    bool fx[NC], fy[NC], fz[NC], fm[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const unsigned b = s_bits[a + SW * k];
        fx[k] = (b & kXN) != 0;
        fy[k] = (b & kYN) != 0;
        fz[k] = (b & kZN) != 0;
        fm[k] = (b & kMasked) != 0;
    }

    // FP32: the lane's per-direction coefficients (q, 1/q, signed C/dV per
    // axis) held in registers for the whole segment where that keeps the
    // resident waves per SIMD (not for 4 or 8 directions per lane); FP64, at
    // its register limit, reads them from LDS
    constexpr bool REGTAB = sizeof(Real) == 4 && NC != 4 && NC != 8;
    Real tq[REGTAB ? NC : 1], tiq[REGTAB ? NC : 1], tcx[REGTAB ? NC : 1], tcy[REGTAB ? NC : 1],
        tcz[REGTAB ? NC : 1];
    if constexpr (REGTAB) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int n = a + SW * k;
            tq[k] = s_tab[n];
            tiq[k] = s_tab[NP + n];
            tcx[k] = s_tab[2 * NP + n];
            tcy[k] = s_tab[3 * NP + n];
            tcz[k] = s_tab[4 * NP + n];
        }
    }

    double lum_acc = 0.0, me_acc = 0.0;
    int nr_acc = 0;

    for (int z = sg.z0; z < sg.z1; ++z) {
        const Real *pl = s_pl + (NBUF == 2 ? ((z - sg.z0) & 1) : 0) * kPlane * P;
        __syncthreads();
        // prefetch the next plane while this one is computed
        const bool more = z + 1 < sg.z1;
        Real qn[NC], hn[kHPG][NC];
        double fln = 0.0;
        int bmn = 0;
        // this plane's four-momentum bookkeeping of the cell (lanes 0..3),
        // read before the prefetch so its wait does not include it
        const long long cidx = (long long)z * pcells + row;
        double dpre = 0.0;
        if (dT0 && a < 4) dpre = dT0[4 * cidx + a];
        // the second stage's base state of this plane, likewise read before
        // the prefetch is issued (FP32; the FP64 kernel has no registers left
        // for it and reads it where it is used)
        constexpr bool IBPRE = STG && sizeof(Real) == 4;
        Real ibv[IBPRE ? NC : 1];
        if constexpr (IBPRE) {
            if (st.Ib) {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const int n = a + SW * k;
                    ibv[k] = (k < NC - 1 || n < N) ? st.Ib[cidx * N + n] : Real(0);
                }
            }
        }
        if (more) {
            load_row(z + 3, row, 0u, qn);
#pragma unroll
            for (int j = 0; j < kHPG; ++j) load_row(z + 1, hrow[j], htest[j], hn[j]);
            fln = load_fluid(z + 1);   // lane 7 re-reads T, unused
            bmn = load_beam(z + 1);
        }
        const bool lum_here = on_lum_xy || (G.lum_axis == 2 && z == (lside ? G.n2 - 1 : 0));
        const bool lum_wave = __ballot(lum_here) != 0;   // wave-uniform

        // ------------------------------------------------------ transport
        Real Is[NC];
        // Each feature flag is 0 (off), 1 (on) or 2 (tested at run time): the
        // common cases get straight-line code over the NC directions, which
        // the compiler can interleave; the rest take the generic variant.
        auto transport = [&](auto tP, auto tM, auto tS, auto tL) {
            constexpr int vP = decltype(tP)::value, vM = decltype(tM)::value;
            constexpr int vS = decltype(tS)::value, vL = decltype(tL)::value;
            const bool doP = vP == 1 || (vP == 2 && plm);
            const bool doM = vM == 1 || (vM == 2 && M.any_mask);
            const bool doS = vS == 1 || (vS == 2 && Istar != nullptr);
            const bool doL = vL == 1 || (vL == 2 && lum_wave);
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int n = a + SW * k;
                const Real Ic = qz[2][k];
                // upwind-ordered neighbours; a direction without motion along
                // an axis has a zero coefficient there, so its branch is
                // irrelevant
                const bool nx = fx[k], ny = fy[k], nz = fz[k];
                // all four axis-0/1 neighbours at fixed offsets, then the upwind order
                const Real xm2 = pl[ox[0] + n], xm1 = pl[ox[1] + n];
                const Real xp1 = pl[ox[2] + n], xp2 = pl[ox[3] + n];
                const Real ym2 = pl[oy[0] + n], ym1 = pl[oy[1] + n];
                const Real yp1 = pl[oy[2] + n], yp2 = pl[oy[3] + n];
                const Real x0 = nx ? xp2 : xm2, x1 = nx ? xp1 : xm1, x3 = nx ? xm1 : xp1;
                const Real y0 = ny ? yp2 : ym2, y1 = ny ? yp1 : ym1, y3 = ny ? ym1 : yp1;
                // upper axis-2 face: the outflow face for motion along +axis 2
                // (upwind cell z), the inflow face otherwise (upwind cell z+1)
                const Real zl = nz ? qz[4][k] : qz[1][k];
                const Real zm = nz ? qz[3][k] : qz[2][k];
                const Real zr = nz ? qz[2][k] : qz[3][k];
                Real Iax, Ibx, Iay, Iby, zup;
                if (doP) {
                    Iax = x1 + half_slope(x0, x1, Ic);
                    Ibx = Ic + half_slope(x1, Ic, x3);
                    Iay = y1 + half_slope(y0, y1, Ic);
                    Iby = Ic + half_slope(y1, Ic, y3);
                    zup = zm + half_slope(zl, zm, zr);
                } else {
                    Iax = x1;
                    Ibx = Ic;
                    Iay = y1;
                    Iby = Ic;
                    zup = zm;
                }
                // inflow (a) and outflow (b) face values along axis 2
                const Real Iaz = nz ? zup : zc[k];
                const Real Ibz = nz ? zc[k] : zup;
                zc[k] = zup;
                // signed coefficients: +-C/dV with the sign of the motion
                const Real cx = REGTAB ? tcx[REGTAB ? k : 0] : s_tab[2 * NP + n];
                const Real cy = REGTAB ? tcy[REGTAB ? k : 0] : s_tab[3 * NP + n];
                const Real cz = REGTAB ? tcz[REGTAB ? k : 0] : s_tab[4 * NP + n];
                const Real dq = fma(cz, Ibz - Iaz, fma(cy, Iby - Iay, cx * (Ibx - Iax)));
                Real Qb = Ic;
                if constexpr (STG) {
                    if (st.Ib) {
                        if constexpr (IBPRE)
                            Qb = Real(st.gI) * Ic + Real(st.gB) * ibv[k];
                        else
                            Qb = Real(st.gI) * Ic +
                                 Real(st.gB) * ((k < NC - 1 || n < N) ? st.Ib[cidx * N + n] : Real(0));
                    }
                }
                const int kt = REGTAB ? k : 0;
                const Real Qs = fma(-dtR, dq, (REGTAB ? tq[kt] : s_tab[n]) * Qb);
                Is[k] = REGTAB ? Qs * tiq[kt] : Qs / s_tab[n];
                if (doM) {
                    const bool msk = fm[k];
                    me_acc -= msk ? (STG ? st.wS : 1.0) * vol * s_dom_all[n] * (double)Qs : 0.0;
                    Is[k] = msk ? Real(0) : Is[k];
                }
                if (doS && (k < NC - 1 || n < N)) Istar[cidx * N + n] = Is[k];
                if (doL) {
                    // energy leaving through the face.  With the signed
                    // coefficients, the face's flux (dA n^a n_0 I_up)/dV is
                    // c Ib when the face is on the outflow side of the cell,
                    // -c Ia when on the inflow side; the outward orientation
                    // of a lower face adds a minus sign
                    double F = 0.0;
                    if (G.lum_axis == 0) F = (double)(nx == (lside == 0) ? cx * Ibx : -(cx * Iax));
                    else if (G.lum_axis == 1) F = (double)(ny == (lside == 0) ? cy * Iby : -(cy * Iay));
                    else F = (double)(nz == (lside == 0) ? cz * Ibz : -(cz * Iaz));
                    lum_acc -= lum_here ? s_dom_all[n] * vol * F : 0.0;
                }
            }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        // (FP64 keeps the generic variant: straight-line FP64 code over six
        // directions does not fit the register file)
        if (sizeof(Real) == 4 && plm && !M.any_mask && !lum_wave) {
            if (Istar)
                transport(I1{}, I0{}, I1{}, I0{});
            else
                transport(I1{}, I0{}, I0{}, I0{});
        } else {
            transport(I2{}, I2{}, I2{}, I2{});
        }

        // ------------------------------------------------------ coupling
        const double u1 = s_fl[cl][0], u2 = s_fl[cl][1], u3 = s_fl[cl][2];
        const double rh = s_fl[cl][3], aa = s_fl[cl][4] * rh, as = s_fl[cl][5] * rh;
        const double Tm = (STG && st.Tb) ? st.gT * s_fl[cl][6] + st.gTb * st.Tb[cidx] : s_fl[cl][6];
        const double u0 = sqrt(1.0 + u1 * u1 + u2 * u2 + u3 * u3);
        const double tau = (aa + as) * dt;
        double Em = 0.0, A1 = 0.0, A2 = 0.0;
        Real kk[NC], gg[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int n = a + SW * k;
            const double dom = s_dom[n];
            const double nb = u0 - fma(u1, s_nh[n], fma(u2, s_nh[NP + n], u3 * s_nh[2 * NP + n]));
            const double dn = fma(nb, tau, n0u);
            // 1/(nb^2 dn); one Newton step suffices for FP32 intensities
            const double r = sizeof(Real) == 4 ? rcp64_1(nb * nb * dn) : rcp64(nb * nb * dn);
            const double r1 = nb * r;                  // 1/(nb dn)
            const double kn = n0u * nb * r1;           // n^0/dn
            const double Iw = (double)Is[k] * (nb * nb * dom);
            Em += Iw;
            A1 = fma(kn, Iw, A1);
            A2 = fma(dom, r1, A2);
            kk[k] = Real(kn);
            gg[k] = Real(nb * dn * r * r);             // 1/(dn nb^3)
        }
        if constexpr (SW == 32) {
            double sp[2] = {Em, A1}, ss[1] = {A2};
            group_sum32_pairs<1, 1>(sp, ss);
            Em = sp[0];
            A1 = sp[1];
            A2 = ss[0] * (dt / kFourPi);
        } else {
            double sf[3] = {Em, A1, A2};
            group_sum_v<SW, 3>(sf);
            Em = sf[0];
            A1 = sf[1];
            A2 = sf[2] * (dt / kFourPi);
        }
        const double B4 = A2 * aa * G.a_rad;
        const double B1 = rh * G.cv * (1.0 - A2 * as);
        const double B0 = A1 - B1 * Tm - (1.0 - A2 * as) * Em;
        int bad = 0;
        const double Tp = quartic_root_fast(B4, B1, B0, bad, Tm);
        const double Ep = Em - rh * G.cv * (Tp - Tm);
        const double Tp2 = Tp * Tp;
        const double S = aa * G.a_rad * Tp2 * Tp2 + as * Ep;
        const Real cS = Real(S * (dt / kFourPi));
        const bool beam_cell = s_beam[cl] != 0;
        Real *dst = Iout + cidx * N;
        Real Ipv[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int n = a + SW * k;
            const Real Ip = fma(kk[k], Is[k], cS * gg[k]);
            Ipv[k] = Ip;
            // (no masked direction anywhere: the select is skipped, wave-uniform)
            Real out = (M.any_mask && fm[k]) ? Real(0) : Ip;
            out = (beam_cell && n == G.beam_angle) ? Real(G.beam_I) : out;
            if (k < NC - 1 || n < N) dst[n] = out;
        }
        if (a == 0) {
            T[cidx] = Tp;
            nr_acc += bad;
        }
        if (dT0) {
            // four-momentum handed to the gas: -n^0 E0 . sum (I+ - I*) (1, n) dOmega
            double sm[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int n = a + SW * k;
                const double dI = (double)(Ipv[k] - Is[k]) * s_dom[n];
                sm[0] += dI;
                sm[1] = fma(dI, s_nh[n], sm[1]);
                sm[2] = fma(dI, s_nh[NP + n], sm[2]);
                sm[3] = fma(dI, s_nh[2 * NP + n], sm[3]);
            }
            if constexpr (SW == 32) {
                double none[1] = {0.0};
                group_sum32_pairs<2, 0>(sm, none);
            } else {
                group_sum_v<SW, 4>(sm);
            }
            if (a < 4) {
                const int al = a;
                dT0[4 * cidx + al] = dpre - (STG ? st.wS : 1.0) * n0u *
                                                (E0[4 * al] * sm[0] + E0[4 * al + 1] * sm[1] +
                                                 E0[4 * al + 2] * sm[2] + E0[4 * al + 3] * sm[3]);
            }
        }
        // single buffer: every group must be done reading plane z first.
        // Double buffer: the other buffer held plane z-1, whose readers have
        // all passed this iteration's first barrier.  The fluid slot of a
        // cell is read only by its own lane group, which wrote it.
        if constexpr (NBUF == 1) __syncthreads();
        if (more) {
            Real *nx = s_pl + (NBUF == 2 ? ((z + 1 - sg.z0) & 1) : 0) * kPlane * P;
            // next plane into LDS straight from the queue and prefetch registers
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int n = a + SW * k;
                nx[o_c + n] = qz[3][k];
#pragma unroll
                for (int j = 0; j < kHPG; ++j) nx[(kTC + kHPG * cl + j) * P + n] = hn[j][k];
                qz[0][k] = qz[1][k];
                qz[1][k] = qz[2][k];
                qz[2][k] = qz[3][k];
                qz[3][k] = qz[4][k];
                qz[4][k] = qn[k];
            }
            if (a < 7) s_fl[cl][a] = fln;
            if (a == 7) s_beam[cl] = bmn;
        }
    }

    // per-block partial sums (fixed order)
    const int wave = threadIdx.x / kWave;
    lum_acc = group_sum<kWave>(lum_acc);
    me_acc = group_sum<kWave>(me_acc);
    nr_acc = group_sum_i<kWave>(nr_acc);
    if (lane == 0) {
        sh_l[wave] = lum_acc;
        sh_m[wave] = me_acc;
        sh_n[wave] = nr_acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double l = 0.0, m = 0.0;
        int r = 0;
        for (int w = 0; w < NW; ++w) {
            l += sh_l[w];
            m += sh_m[w];
            r += sh_n[w];
        }
        partials[2 * blockIdx.x] = l;
        partials[2 * blockIdx.x + 1] = m;
        nr_partial[blockIdx.x] = r;
    }
}

template <typename Real, int SW, int NC, bool STG = false>
int launch_one(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
               const double *rho, const double *u, const double *ka, const double *ks,
               double dt, double *dT0, Real *Istar, const Partials &P,
               const MStage<Real> &st = MStage<Real>{}) {
    const MarchInfo &M = g->march;
    if (ensure_dynamic_lds(reinterpret_cast<const void *>(&k_march<Real, SW, NC, STG>), M.lds) !=
        RT_OK)
        return RT_EDEVICE;
    hipLaunchKernelGGL((k_march<Real, SW, NC, STG>), dim3(M.grid), dim3(kTC * SW), M.lds, s,
                       g->dg, M, static_cast<const Real *>(Iin), static_cast<Real *>(Iout), T, rho,
                       u, ka, ks, dt, dT0, P.sums, P.noroot, Istar, st);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

// The two-stage step on the tiled path (instantiated for 32 lanes x 6
// directions): stage 1 into the grid's stage buffers, stage 2 from them and
// from I_in, T into I_out, T; each stage's luminosity counts dt/2.
template <typename Real>
int march_rk2_t(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                const double *rho, const double *u, const double *ka, const double *ks,
                double dt, double *dT0, double *lum, const Partials &P) {
    const size_t ncell = (size_t)g->dg.n0 * g->dg.n1 * g->dg.n2;
    if (hipMemcpyAsync(g->stage_T, T, ncell * sizeof(double), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return RT_EDEVICE;
    const MStage<Real> s1{nullptr, nullptr, 1.0, 0.0, 1.0, 1.0, 0.0, 0.5};
    int rc = launch_one<Real, 32, 6, true>(g, s, Iin, g->stage_I, g->stage_T, rho, u, ka, ks, dt,
                                           dT0, nullptr, P, s1);
    if (rc == RT_OK) rc = launch_finalize(g, s, g->march.grid, 0.5 * dt, lum, P);
    if (rc != RT_OK) return rc;
    const MStage<Real> s2{static_cast<const Real *>(Iin), g->stage_T, 0.5, 0.5, 0.5, 0.5, 0.5, 1.0};
    rc = launch_one<Real, 32, 6, true>(g, s, g->stage_I, Iout, T, rho, u, ka, ks, dt, dT0, nullptr,
                                       P, s2);
    if (rc == RT_OK) rc = launch_finalize(g, s, g->march.grid, 0.5 * dt, lum, P);
    return rc;
}

}  // namespace

bool march_rk2_config(int sw, int nc) { return sw == 32 && nc == 6; }

int launch_march_rk2(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                     const double *rho, const double *u, const double *ka, const double *ks,
                     double dt, double *dT0, double *lum, const Partials &P) {
    if (!march_rk2_config(g->march.sw, g->march.nc)) return RT_EINVAL;
    if (g->precision == RT_F32)
        return march_rk2_t<float>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
    return march_rk2_t<double>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
}

// Lane-group width and directions per lane for each supported direction count.
bool march_config(int precision, int nang, int &sw, int &nc) {
    // instantiated (lane-group width, directions per lane) pairs
    static const int f32[][2] = {{16, 1}, {16, 3}, {16, 6}, {32, 3}, {32, 4}, {32, 6}, {32, 8}};
    static const int f64[][2] = {{16, 1}, {16, 3}, {16, 6}, {32, 3}, {32, 4}, {32, 6}};
    const int (*tab)[2] = precision == RT_F32 ? f32 : f64;
    const int ntab = precision == RT_F32 ? 7 : 6;
    // smallest group width whose directions-per-lane fits the register
    // budget; directions per lane must be exactly ceil(nang / width), since
    // the kernel lets only the last chunk of a lane run past nang
    const int budget = 6;
    for (int w : {16, 32}) {
        const int need = (nang + w - 1) / w;
        if (need > budget) continue;
        for (int i = 0; i < ntab; ++i)
            if (tab[i][0] == w && tab[i][1] == need) {
                sw = w;
                nc = need;
                return true;
            }
    }
    return false;
}

// LDS stride of one plane cell: the direction count rounded so that the
// lane groups of a wavefront, which read neighbouring plane cells, start on
// different LDS banks
int march_pstride(int precision, int nang) {
    const int per_bank_row = precision == RT_F32 ? 64 : 32;   // 256-byte rows
    const int quarter = per_bank_row / 4;
    int p = (nang + quarter - 1) / quarter * quarter;
    if ((p / quarter) % 2 == 0) p += quarter;
    return p;
}

size_t march_lds_bytes(int precision, int nang, int np) {
    const size_t real = precision == RT_F32 ? 4 : 8;
    const size_t nbuf = precision == RT_F32 ? 2 : 1;   // as NBUF in k_march
    return (size_t)np * (5 * 8 + 5 * real + 1) +
           nbuf * kPlane * march_pstride(precision, np) * real;
}

int launch_march(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                 const double *rho, const double *u, const double *ka, const double *ks,
                 double dt, double *dT0, void *Istar, const Partials &P) {
    const MarchInfo &M = g->march;
#define RT_CASE(R, SW, NC)                                                                    \
    if (M.sw == SW && M.nc == NC)                                                             \
        return launch_one<R, SW, NC>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0,          \
                                     static_cast<R *>(Istar), P);
    if (g->precision == RT_F32) {
        RT_CASE(float, 16, 1)
        RT_CASE(float, 16, 3)
        RT_CASE(float, 16, 6)
        RT_CASE(float, 32, 3)
        RT_CASE(float, 32, 4)
        RT_CASE(float, 32, 6)
        RT_CASE(float, 32, 8)
    } else {
        RT_CASE(double, 16, 1)
        RT_CASE(double, 16, 3)
        RT_CASE(double, 16, 6)
        RT_CASE(double, 32, 3)
        RT_CASE(double, 32, 4)
        RT_CASE(double, 32, 6)
    }
#undef RT_CASE
    return RT_EINVAL;
}

}  // namespace rt
