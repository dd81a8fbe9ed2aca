// Adjoint of the transport for geometry that does not depend on axis 2
// (Sec. 2.3-2.4 reversed; the stationary, axisymmetric Kerr-Schild
// spacetime in spherical coordinates with axis 2 = phi): every geometry
// table of a cell column (i, j) is the same for all of its cells.
//
// dJ/dI of a cell is the general gather's (k_adjoint.hip): psi q, then per
// axis the four faces whose upwind PLM value depends on the cell (faces
// x-3/2 .. x+3/2, each only for the motion sign that puts the cell in its
// upwind stencil), then the angular edges whose upwind side is the
// direction itself -- formed with the shared helpers of k_adj_common.h in
// the same order, so both kernels give bit-identical results.
//
// Mapping (gfx950): one 64-lane wavefront marches one column segment along
// axis 2 for one 64-direction chunk (the transport adjoint has no sums over
// directions, so a row of up to six chunks splits over waves; the waves of
// one column run in neighbouring workgroups, so they share its rows in L2).
//   * the column's geometry per direction -- q, the eight axis-0/1 face
//     coefficients (faces i-1 .. i+2 and j-1 .. j+2), the axis-2
//     coefficient, packed face/ghost/mask flags -- is loaded once per
//     segment into registers; the neighbour cells' 1/dV are scalars;
//   * I and psi of the column come from five-plane register queues (each
//     plane read from HBM once per segment, the next one loaded while the
//     current one is computed);
//   * with FP32 intensities the next plane's sixteen axis-0/1 neighbour rows
//     (I and psi, two columns each way) and the column's full psi row (every
//     direction, for the angular-edge gather; double-buffered) go straight
//     from HBM/L2 into a per-wave LDS buffer by global_load_lds once the
//     current plane's axis-0/1 terms have read them, so they arrive behind
//     the axis-2 and angular terms; in FP64 they are loaded into registers
//     one axis at a time and the psi row is staged through registers;
//   * workgroup order as the forward column kernel: four neighbouring
//     columns per workgroup, bands of 16 rows along axis 1, XCD-aware.
#include <hip/hip_runtime.h>

#include "k_adj_common.h"

namespace rt {
namespace {

constexpr int kAcBlock = 256;
constexpr int kAcWaves = kAcBlock / kWave;
constexpr int kAcBand = 16;               // rows along axis 1 of a band of workgroups
constexpr int kAcMaxAng = 6 * kWave;      // as the forward column kernel

// flag word of one direction of a column: for axis a = 0, 1 and face f =
// 0..3 (faces at offsets -1 .. +2 from the cell's lower face) bit 8a + 2f
// is set when the face contributes with motion along +axis a, bit 8a + 2f + 1
// with motion along -axis a; the axis-2 motion sign; the mask; and the
// neighbour slots (x-2, x-1, x+1, x+2, y-2, y-1, y+1, y+2) whose intensity is
// a zero vacuum ghost
constexpr unsigned kAzP = 1u << 16, kAzN = 1u << 17, kAMsk = 1u << 18;
constexpr int kAGhostShift = 20;

// element n of a row at a wave-uniform address: a scalar base plus a 32-bit
// lane byte offset (the global_load "saddr" form, one VGPR per offset)
template <typename Real>
__device__ __forceinline__ const Real *at_lane(const Real *row, unsigned n) {
    return reinterpret_cast<const Real *>(reinterpret_cast<const char *>(row) +
                                          (unsigned)(n * sizeof(Real)));
}

__device__ __forceinline__ void acol_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the four faces of one axis for one direction: fb holds the axis's eight
// face bits, fon the luminosity faces (bit f, wave-uniform), seed the
// luminosity seed of the direction; v, ps, iv are I, psi and 1/dV at offsets
// -2 .. +2; C the face coefficients.  Branch-free: every face term is
// formed and kept by a select where the face contributes, so the sum is
// bit-identical to the general gather's conditional additions.
template <typename Real>
__device__ __forceinline__ void adj_axis(Real &lam, const Real (&v)[5], const Real (&ps)[5],
                                         const Real (&iv)[5], const Real (&C)[4], unsigned fb,
                                         unsigned fon, Real seed, bool plm, Real dtR) {
    // limiter partials of the upwind cells u = -1, 0, +1 (index u + 1)
    Real hx[3], hy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        hx[k] = Real(0);
        hy[k] = Real(0);
        if (plm) half_slope_partials(v[k], v[k + 1], v[k + 2], hx[k], hy[k]);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const bool P = (fb >> (2 * f)) & 1u, Nn = (fb >> (2 * f + 1)) & 1u;
        const int fo = f - 1;
        const int u = P ? fo - 1 : fo;
        // index u + 1 of the limiter partials, for either sign (the sign
        // that would leave -1 .. 1 never has its bit set)
        const int iP = fo < 0 ? 0 : fo, iN = fo + 1 > 2 ? 2 : fo + 1;
        Real dh = Real(0);
        if (plm) dh = dh_at(u, P ? hx[iP] : hx[iN], P ? hy[iP] : hy[iN]);
        const Real d = face_weight(u == 0, P, plm, dh);
        Real lF = face_adjoint(dtR, ps[fo + 2], iv[fo + 2], ps[fo + 1], iv[fo + 1]);
        if ((fon >> f) & 1u) lF += seed;
        Real t = lam;
        face_add(t, lF, C[f], d);
        lam = (P || Nn) ? t : lam;
    }
}

template <typename Real, int NCW>
constexpr int acol_waves() {
    return sizeof(Real) == 4 && NCW == 1 ? 3 : 2;
}
template <typename Real, int NCW, bool DMA>
__global__ __launch_bounds__(kAcBlock) __attribute__((amdgpu_waves_per_eu(acol_waves<Real, NCW>()))) void k_adj_column(DevGrid G, ColumnInfo CI, int nsplit,
                                                         int ostride, int wave_lds,
                                                         const Real *__restrict__ Iin,
                                                         const Real *__restrict__ psi, double dt,
                                                         double lum_weight, Real *__restrict__ lam) {
    const int lane = threadIdx.x % kWave;
    // wave-uniform (scalar registers): the column and every row address
    // derived from it, so loads take a scalar base plus a lane offset
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int N = G.nang;
    const int nchT = (N + kWave - 1) / kWave;
    __shared__ Real s_iom[kAcMaxAng];
    extern __shared__ __align__(16) unsigned char s_dyn[];
    // per wave: two psi rows of the column [2][ostride], then (DMA) the next
    // plane's neighbour rows [16][NCW][64] (I rows 0..7, psi rows 8..15)
    Real *s_row = reinterpret_cast<Real *>(s_dyn) + (size_t)wave * wave_lds;
    Real *s_nb = s_row + 2 * ostride;
    for (int k = threadIdx.x; k < N; k += kAcBlock) s_iom[k] = Real(1.0 / G.domega[k]);

    // XCD-aware logical block; the direction slices of a column are
    // neighbouring logical blocks
    const int per = gridDim.x / 8;
    const int lb = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    const int sp = lb % nsplit;
    const int logical = lb / nsplit;
    const int cb = sp * NCW;   // first chunk of this wave's slice
    const long long pcells = (long long)G.n0 * G.n1;
    const int nq = (G.n0 + kAcWaves - 1) / kAcWaves;
    const long long per_seg = (long long)nq * G.n1;
    const int seg = (int)(logical / per_seg);
    const int r = (int)(logical % per_seg);
    const int nband = (G.n1 + kAcBand - 1) / kAcBand;
    const int band = min(r / (nq * kAcBand), nband - 1);
    const int h = min(kAcBand, G.n1 - band * kAcBand);
    const int t = r - band * nq * kAcBand;
    int i = (t / h) * kAcWaves + wave, j = band * kAcBand + t % h, z0 = 0, z1 = 0;
    const bool active = seg < CI.nseg && i < G.n0 && cb < nchT;
    if (active) {
        z0 = seg * CI.seglen;
        z1 = min(G.n2, z0 + CI.seglen);
    } else {
        i = 0;
        j = 0;
    }
    Cell x;
    x.i = i;
    x.j = j;
    x.k = 0;
    x.c = (long long)j * G.n0 + i;
    x.gc = (G.g1 > 1 ? j : 0) * G.g0 + (G.g0 > 1 ? i : 0);
    const Real *q = static_cast<const Real *>(G.q);
    const Real *invV = static_cast<const Real *>(G.invV);
    const Real *vw = static_cast<const Real *>(G.vw);
    const Real ivol = invV[x.gc];
    const bool plm = G.recon == RT_RECON_PLM;
    const Real dtR = Real(dt);
    const int E = G.nedge;

    // ------------------------------------------------ column geometry, once
    // neighbour columns (slot k = x-2, x-1, x+1, x+2, y-2, y-1, y+1, y+2),
    // the faces beyond which a vacuum ghost sits (-1: active or periodic
    // neighbour) and the neighbours' 1/dV (zero outside a non-periodic
    // boundary, where psi is zero too)
    int ncol[8], gface[8];
    Real ivn[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int a = k / 4;
        const int o = (k % 4) < 2 ? (k % 4) - 2 : (k % 4) - 1;
        const int coord = a == 0 ? i : j;
        const int len = a == 0 ? G.n0 : G.n1;
        int idx = coord + o;
        gface[k] = -1;
        bool inside = true;
        if (idx < 0 || idx >= len) {
            const int side = idx < 0 ? 0 : 1;
            if (G.bc[a][side] == RT_BC_PERIODIC) {
                idx = ((idx % len) + len) % len;
            } else {
                inside = false;
                gface[k] = face_geo(G, a, side ? len : 0, x);
                idx = side ? len - 1 : 0;
            }
        }
        ncol[k] = a == 0 ? j * G.n0 + idx : idx * G.n0 + i;
        const int gstr = a == 0 ? (G.g0 > 1 ? 1 : 0) : (G.g1 > 1 ? G.g0 : 0);
        ivn[k] = inside ? invV[x.gc + (idx - coord) * gstr] : Real(0);
    }
    // whether a vacuum ghost borders the column along axis 0 or 1 (wave-
    // uniform: most columns have none and skip the per-direction zeroing)
    const bool ghost_x = gface[0] >= 0 || gface[1] >= 0 || gface[2] >= 0 || gface[3] >= 0;
    const bool ghost_y = gface[4] >= 0 || gface[5] >= 0 || gface[6] >= 0 || gface[7] >= 0;
    // faces of axes 0 and 1: geometry rows, which sign may contribute, the
    // luminosity faces
    int fg[2][4];
    unsigned pv[2] = {0u, 0u}, nv[2] = {0u, 0u}, fon[2] = {0u, 0u};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int coord = a == 0 ? i : j;
        const int len = a == 0 ? G.n0 : G.n1;
        const bool periodic = G.bc[a][0] == RT_BC_PERIODIC;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int fo = f - 1;
            const int Fraw = coord + fo;
            const bool fvalid = periodic || (Fraw >= 0 && Fraw <= len);
            const int F = periodic ? ((Fraw % len) + len) % len : Fraw;
            fg[a][f] = face_geo(G, a, fvalid ? F : 0, x);
            // upwind cell fo-1 (motion along +a) or fo (along -a): within
            // -1 .. 1 of the cell and not a ghost
            const int up = coord + fo - 1, un = coord + fo;
            if (fvalid && fo >= 0 && (periodic || (up >= 0 && up < len))) pv[a] |= 1u << f;
            if (fvalid && fo <= 1 && (periodic || (un >= 0 && un < len))) nv[a] |= 1u << f;
            if (a == G.lum_axis && fvalid &&
                (periodic ? F == 0 : (G.lum_side == 1 ? F == len : F == 0)))
                fon[a] |= 1u << f;
        }
    }
    const int fz = face_geo(G, 2, 0, x);   // every axis-2 face of the column
    Real gq[NCW], cf[2][4][NCW], czz[NCW];
    unsigned fl[NCW];
#pragma unroll
    for (int ch = 0; ch < NCW; ++ch) {
        const int n = lane + kWave * (cb + ch);
        const int m = n < N ? n : N - 1;
        gq[ch] = q[(size_t)x.gc * N + m];
        unsigned f = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const Real *C = static_cast<const Real *>(G.C[a]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                cf[a][k][ch] = C[(size_t)fg[a][k] * N + m];
                const int s = G.sgn[a][(size_t)fg[a][k] * N + m];
                if (s > 0 && ((pv[a] >> k) & 1u)) f |= 1u << (8 * a + 2 * k);
                if (s < 0 && ((nv[a] >> k) & 1u)) f |= 1u << (8 * a + 2 * k + 1);
            }
        }
        czz[ch] = static_cast<const Real *>(G.C[2])[(size_t)fz * N + m];
        const int sz = G.sgn[2][(size_t)fz * N + m];
        f |= sz > 0 ? kAzP : (sz < 0 ? kAzN : 0u);
        if (G.mask[(size_t)x.gc * N + m]) f |= kAMsk;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (gface[k] < 0) continue;
            // ghost beyond a lower (slots 0, 1) or upper face: the edge cell
            // for directions leaving through it, zero for directions entering
            const int s = G.sgn[k / 4][(size_t)gface[k] * N + m];
            const bool out = (k % 4) < 2 ? (s < 0) : (s > 0);
            if (!out) f |= 1u << (kAGhostShift + k);
        }
        fl[ch] = f;
    }
    // the lane's directions' angular edges, kept in registers for the whole
    // march: the edge's other direction and its signed weight (zero for a
    // slot past the direction's edges or whose upwind side is the other
    // direction: the slot then adds nothing)
    const Real *vwrow = vw + (size_t)x.gc * E * 2;
    int pe[kMaxNbr][NCW];
    Real sw[kMaxNbr][NCW], iom[NCW];
#pragma unroll
    for (int ch = 0; ch < NCW; ++ch) {
        const int m = min(lane + kWave * (cb + ch), N - 1);
        iom[ch] = Real(1.0 / G.domega[m]);
#pragma unroll
        for (int s = 0; s < kMaxNbr; ++s) {
            pe[s][ch] = m;
            sw[s][ch] = Real(0);
            const int e = G.has_edges ? G.adj_e[m * kMaxNbr + s] : -1;
            if (e < 0) continue;
            const Real vv = vwrow[2 * e], ww = vwrow[2 * e + 1];
            const bool is_lo = G.adj_s[m * kMaxNbr + s] > 0;
            const bool up = is_lo ? vv > Real(0) : vv < Real(0);
            pe[s][ch] = is_lo ? G.edge_hi[e] : G.edge_lo[e];
            if (up) sw[s][ch] = edge_weight(dtR, ww, is_lo);
        }
    }
    // luminosity seed of the lane's directions (used on luminosity faces)
    Real seed[NCW];
#pragma unroll
    for (int ch = 0; ch < NCW; ++ch)
        seed[ch] = lum_seed<Real>(G, lum_weight, dt, min(lane + kWave * (cb + ch), N - 1));
    __syncthreads();   // s_iom
    if (!active) return;

    const bool zper = G.bc[2][0] == RT_BC_PERIODIC;
    const int mycol = (int)x.c;
    // plane pz of the column, I and psi as stored (the wrapped or edge
    // plane), and what the axis-2 boundary condition makes of them: I keeps
    // the edge cell only for directions leaving through that face (`need`
    // bit; 0: kept); psi keeps the edge plane, whose 1/dV there is zero (as
    // in the general gather).  The condition is applied where a plane enters
    // the queue, so a prefetched plane is not waited for when it is issued.
    auto load_raw = [&](int pz, Real (&dI)[NCW], Real (&dP)[NCW], unsigned &need) {
        long long zz = pz;
        need = 0;
        if (pz < 0 || pz >= G.n2) {
            const int side = pz < 0 ? 0 : 1;
            if (zper) {
                zz = ((pz % G.n2) + G.n2) % G.n2;
            } else {
                need = side ? kAzP : kAzN;
                zz = side ? G.n2 - 1 : 0;
            }
        }
        const Real *srcI = Iin + (zz * pcells + mycol) * N;
        const Real *srcP = psi + (zz * pcells + mycol) * N;
#pragma unroll
        for (int ch = 0; ch < NCW; ++ch) {
            const unsigned n = (unsigned)min(lane + kWave * (cb + ch), N - 1);
            dI[ch] = *at_lane(srcI, n);
            dP[ch] = *at_lane(srcP, n);
        }
    };
    auto enqueue = [&](const Real (&dI)[NCW], const Real (&dP)[NCW], unsigned need,
                       Real (&qI)[NCW], Real (&qP)[NCW]) {
#pragma unroll
        for (int ch = 0; ch < NCW; ++ch) {
            qI[ch] = (need == 0 || (fl[ch] & need)) ? dI[ch] : Real(0);
            qP[ch] = dP[ch];   // outside: the edge plane, times 1/dV = 0
        }
    };
    // DMA: the sixteen neighbour rows of plane pz (this wave's chunks) and
    // the column's full psi row into buffer `row`; each lane moves one value
    // per (row, chunk); lanes past the row re-read its last entry (never used)
    auto dma_plane = [&](int pz, Real *row) {
        if constexpr (DMA) {
            const Real *bI = Iin + (long long)pz * pcells * N;
            const Real *bP = psi + (long long)pz * pcells * N;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const Real *rI = bI + (long long)ncol[k] * N;
                const Real *rP = bP + (long long)ncol[k] * N;
#pragma unroll
                for (int ch = 0; ch < NCW; ++ch) {
                    const unsigned n = (unsigned)min(lane + kWave * (cb + ch), N - 1);
                    __builtin_amdgcn_global_load_lds(
                        at_lane(rI, n), (__attribute__((address_space(3))) void *)(s_nb + (k * NCW + ch) * kWave),
                        4, 0, 0);
                    __builtin_amdgcn_global_load_lds(
                        at_lane(rP, n),
                        (__attribute__((address_space(3))) void *)(s_nb + ((8 + k) * NCW + ch) * kWave), 4,
                        0, 0);
                }
            }
            if (G.has_edges) {
                const Real *src = bP + (long long)mycol * N;
                for (int c = 0; c < nchT; ++c)
                    __builtin_amdgcn_global_load_lds(
                        at_lane(src, (unsigned)min(lane + kWave * c, N - 1)),
                        (__attribute__((address_space(3))) void *)(row + kWave * c), 4, 0, 0);
            }
        }
    };
    // register path: the four neighbour rows of axis a at plane pz
    auto load_axis = [&](int pz, int a, Real (&dI)[4][NCW], Real (&dP)[4][NCW]) {
        const Real *bI = Iin + (long long)pz * pcells * N;
        const Real *bP = psi + (long long)pz * pcells * N;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * a + kk;
#pragma unroll
            for (int ch = 0; ch < NCW; ++ch) {
                const int n = min(lane + kWave * (cb + ch), N - 1);
                dI[kk][ch] = bI[(long long)ncol[k] * N + n];
                dP[kk][ch] = bP[(long long)ncol[k] * N + n];
            }
        }
    };

    Real qi[5][NCW], qp[5][NCW];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        Real dI[NCW], dP[NCW];
        unsigned need;
        load_raw(z0 - 2 + p, dI, dP, need);
        enqueue(dI, dP, need, qi[p], qp[p]);
    }
    if constexpr (DMA) dma_plane(z0, s_row);

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;
        Real *own = s_row + ((z - z0) & 1) * ostride;
        if constexpr (DMA) {
            // this plane's rows have landed (the wave's own loads: vmcnt
            // reaches zero)
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        } else {
            if (G.has_edges) {
                const Real *src = psi + ((long long)z * pcells + mycol) * N;
                for (int c = 0; c < nchT; ++c) {
                    const int n = lane + kWave * c;
                    if (n < N) own[n] = src[n];
                }
                acol_wave_sync();
            }
        }
        // the column's plane z+3 while this one is computed
        Real ni[NCW], np[NCW];
        unsigned nneed = 0;
        if (more) load_raw(z + 3, ni, np, nneed);
        // axis-2 faces of this plane: which sign may contribute, the
        // luminosity faces, 1/dV at offsets -2 .. +2
        unsigned zv = 0, zfon = 0;
        Real ivz[5];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int fo = f - 1;
            const int Fraw = z + fo;
            const bool fvalid = zper || (Fraw >= 0 && Fraw <= G.n2);
            const int F = zper ? ((Fraw % G.n2) + G.n2) % G.n2 : Fraw;
            const int up = z + fo - 1, un = z + fo;
            if (fvalid && fo >= 0 && (zper || (up >= 0 && up < G.n2))) zv |= 1u << (2 * f);
            if (fvalid && fo <= 1 && (zper || (un >= 0 && un < G.n2))) zv |= 1u << (2 * f + 1);
            if (G.lum_axis == 2 && fvalid && (zper ? F == 0 : (G.lum_side == 1 ? F == G.n2 : F == 0)))
                zfon |= 1u << f;
        }
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            const int zz = z + o - 2;
            ivz[o] = (zper || (zz >= 0 && zz < G.n2)) ? ivol : Real(0);
        }

        Real acc[NCW];
#pragma unroll
        for (int ch = 0; ch < NCW; ++ch)
            acc[ch] = (fl[ch] & kAMsk) ? Real(0) : qp[2][ch] * gq[ch];
        // axes 0 and 1
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            Real nI[4][NCW], nP[4][NCW];
            if constexpr (DMA) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * a + kk;
#pragma unroll
                    for (int ch = 0; ch < NCW; ++ch) {
                        nI[kk][ch] = s_nb[(k * NCW + ch) * kWave + lane];
                        nP[kk][ch] = s_nb[((8 + k) * NCW + ch) * kWave + lane];
                    }
                }
            } else {
                load_axis(z, a, nI, nP);
            }
#pragma unroll
            for (int ch = 0; ch < NCW; ++ch) {
                const int n = min(lane + kWave * (cb + ch), N - 1);
                const unsigned f = fl[ch];
                Real v[5], ps[5], iv[5], C[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * a + kk;
                    const int o = kk < 2 ? kk : kk + 1;
                    v[o] = nI[kk][ch];
                    ps[o] = nP[kk][ch];   // outside: the edge row, times 1/dV = 0
                    iv[o] = ivn[k];
                    C[kk] = cf[a][kk][ch];
                }
                if (a == 0 ? ghost_x : ghost_y) {
                    // the flag tests are formed here, not kept as lane masks
                    // across the march
                    unsigned fg = f;
                    asm volatile("" : "+v"(fg));
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
                        if (fg & (1u << (kAGhostShift + 4 * a + kk))) v[kk < 2 ? kk : kk + 1] = Real(0);
                }
                v[2] = qi[2][ch];
                ps[2] = qp[2][ch];
                iv[2] = ivol;
                adj_axis(acc[ch], v, ps, iv, C, (f >> (8 * a)) & 0xffu, fon[a], seed[ch], plm, dtR);
            }
        }
        if constexpr (DMA) {
            if (more) {
                // every LDS read of this plane's rows has returned before the
                // next plane's rows are written over them
                __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
                dma_plane(z + 1, s_row + ((z + 1 - z0) & 1) * ostride);
            }
        }
        // axis 2 and the angular edges
        Real *dst = lam + ((long long)z * pcells + x.c) * N;
#pragma unroll
        for (int ch = 0; ch < NCW; ++ch) {
            const int n = lane + kWave * (cb + ch);
            const int m = min(n, N - 1);
            const unsigned f = fl[ch];
            {
                const Real v[5] = {qi[0][ch], qi[1][ch], qi[2][ch], qi[3][ch], qi[4][ch]};
                const Real ps[5] = {qp[0][ch], qp[1][ch], qp[2][ch], qp[3][ch], qp[4][ch]};
                const Real C[4] = {czz[ch], czz[ch], czz[ch], czz[ch]};
                const unsigned fb = (f & kAzP ? (zv & 0x55u) : 0u) | (f & kAzN ? (zv & 0xAAu) : 0u);
                adj_axis(acc[ch], v, ps, ivz, C, fb, zfon, seed[ch], plm, dtR);
            }
            if (G.has_edges) {
                // branch-free over the six slots (an unused slot adds 0)
                const Real a_n = own[m] * iom[ch];
#pragma unroll
                for (int s = 0; s < kMaxNbr; ++s)
                    edge_add(acc[ch], a_n, own[pe[s][ch]], s_iom[pe[s][ch]], sw[s][ch]);
            }
            if (n < N) dst[n] = acc[ch];
        }
        if (!DMA && G.has_edges) acol_wave_sync();   // own row read before it is rewritten
#pragma unroll
        for (int ch = 0; ch < NCW; ++ch) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                qi[p][ch] = qi[p + 1][ch];
                qp[p][ch] = qp[p + 1][ch];
            }
        }
        if (more) enqueue(ni, np, nneed, qi[4], qp[4]);
    }
}

template <typename Real, int NCW, bool DMA>
int launch_acol(rt_grid *g, hipStream_t s, const Real *Iin, const Real *psi, double dt,
                double lum_weight, Real *lam, int nsplit) {
    const ColumnInfo &CI = g->column;
    const DevGrid &G = g->dg;
    const int nchT = (G.nang + kWave - 1) / kWave;
    if (nchT * kWave > kAcMaxAng) return RT_EINVAL;
    const int ostride = kWave * nchT;
    const int wave_lds = 2 * ostride + (DMA ? 16 * NCW * kWave : 0);
    const size_t lds = (size_t)kAcWaves * wave_lds * sizeof(Real);
    if (lds > 64 * 1024) return RT_EINVAL;
    const long long blocks =
        (long long)((G.n0 + kAcWaves - 1) / kAcWaves) * G.n1 * CI.nseg * nsplit;
    if (blocks >= (1LL << 30)) return RT_EINVAL;
    const int grid = (int)((blocks + 7) / 8 * 8);
    hipLaunchKernelGGL((k_adj_column<Real, NCW, DMA>), dim3(grid), dim3(kAcBlock), lds, s, G, CI,
                       nsplit, ostride, wave_lds, Iin, psi, dt, lum_weight, lam);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

template <typename Real>
int launch_acol_t(rt_grid *g, hipStream_t s, const void *Iin, const void *psi, double dt,
                  double lum_weight, void *lam) {
    const int nch = (g->dg.nang + kWave - 1) / kWave;
    // one direction chunk per wave: the fewest registers (FP32 90 VGPRs,
    // against 160 with two chunks and 197 with three) and the most resident
    // waves outweigh the per-wave work repeated for each chunk (the plane
    // flags, the column's full psi row): 256 x 128 x 256 x 362 adjoint step
    // 81.9 ms against 93.6 (two) and 86.5 (three)
    const int cmax = 1;
    const int nsplit = (nch + cmax - 1) / cmax;
    const int ncw = (nch + nsplit - 1) / nsplit;
    const Real *in = static_cast<const Real *>(Iin);
    const Real *ps = static_cast<const Real *>(psi);
    Real *out = static_cast<Real *>(lam);
    constexpr bool dma = sizeof(Real) == 4;
    if (ncw != 1) return RT_EINVAL;
    return launch_acol<Real, 1, dma>(g, s, in, ps, dt, lum_weight, out, nsplit);
}

}  // namespace

int launch_adj_column(rt_grid *g, hipStream_t s, const void *Iin, const void *psi, double dt,
                      double lum_weight, void *lam) {
    if (g->precision == RT_F32) return launch_acol_t<float>(g, s, Iin, psi, dt, lum_weight, lam);
    return launch_acol_t<double>(g, s, Iin, psi, dt, lum_weight, lam);
}

}  // namespace rt
