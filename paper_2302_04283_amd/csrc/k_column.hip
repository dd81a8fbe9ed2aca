// Fused radiation step for geometry that does not depend on axis 2 (e.g. the
// stationary, axisymmetric Kerr-Schild spacetime in spherical coordinates,
// with axis 2 = phi; paper Sec. 2.1-2.2): every geometry table of a cell
// column (i, j) -- face coefficients, q, signs, mask, angular-edge weights --
// is the same for all of its cells along axis 2.
//
// Mapping (gfx950): one 64-lane wavefront marches one column segment along
// axis 2; lane l handles directions l, l+64, ... (NCH chunks), so the
// coupling's per-cell FP64 angle sums stay wavefront reductions.
//   * the column's geometry is loaded once per segment into registers
//     (q and the five face coefficients per direction, sign/mask/ghost flags
//     packed in one word) and, with FP32 intensities, its angular-edge
//     weights into LDS;
//   * axis-2 neighbours come from a four-plane register queue (each plane
//     of the column is read from HBM once per segment; the next plane is
//     loaded while the current one is computed), and the axis-2 face flux
//     of a plane is carried to the next plane, so the plane below is not
//     needed;
//   * axis-0/1 neighbour rows (two columns each way for PLM): with FP32
//     intensities the next plane's eight rows are loaded into registers as
//     soon as the current plane's transport has read them, so their latency
//     hides behind the angular fluxes and the coupling (except at four
//     chunks, where those registers would cost a resident wave); otherwise
//     they are loaded one axis at a time;
//   * the cell's own row is staged in LDS for the angular-edge gather;
//   * workgroups are dispatched round-robin over the 8 XCDs; the logical
//     order gives each XCD a contiguous band of columns, so neighbour
//     columns marching at the same time share an L2.
// The per-direction arithmetic is the general kernel's (same expressions,
// same order), so both give bit-identical results.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "k_transport.h"

namespace rt {
namespace {

constexpr int kColBlock = 256;
constexpr int kColBand = 16;            // rows along axis 1 of a band of workgroups
// resident waves per SIMD the register allocation is held to: the column's
// geometry and plane queue live in registers, about 25 VGPRs per direction
// chunk in FP32 and 40 in FP64 on top of the coupling's working set
template <typename Real, int NCH, bool TAU = false>
constexpr int col_waves() {
    // (the optical-depth-aware flux's per-direction terms take two waves' worth)
    return TAU ? 2 : (sizeof(Real) == 4 ? (NCH <= 1 ? 4 : (NCH <= 3 ? 3 : 2)) : (NCH <= 2 ? 3 : 2));
}
constexpr int kColWaves = kColBlock / kWave;
// Direction tables staged once per workgroup (byte offsets into dynamic
// LDS): unit vectors by component with a compile-time stride nhs (the
// instantiation's direction slots, so one address serves all three), solid
// angles, and with MAPR the candidate planes' inverse matrices and the edge
// midpoint offsets [E][4] (intensity precision); then the edge records
// [N][6] (not with the per-column edge table), the MAPR neighbour lists and
// neighbour counts [N].  The matrices and neighbour lists are component-major
// in FP32, [24][nhs] and [6][nhs], so a wave's reads of one entry are
// consecutive; FP64 keeps the direction-major [N][24] and [N][6] (the
// padded copies would not fit beside four columns' rows at 162 directions).
// With angular PLM (latitude-longitude grids) each edge's outer stencil
// directions [E] and [E] follow.
struct ColTab {
    size_t nhat, dom, minv, md, adj, mnb, mcnt, ell, err, bytes;
};
__host__ __device__ inline ColTab col_tab(int N, int E, int nhs, int real, bool adj, bool mapr,
                                          bool aplm) {
    ColTab t{};
    const size_t nm = real == 4 ? nhs : N;   // rows of the MAPR tables
    t.nhat = 0;
    t.dom = t.nhat + (size_t)3 * nhs * sizeof(double);
    t.minv = t.dom + (size_t)N * sizeof(double);
    t.md = t.minv + (mapr ? nm * kMaxNbr * 4 * real : 0);
    t.adj = t.md + (mapr ? (size_t)E * 4 * real : 0);
    t.mnb = t.adj + (adj ? (size_t)N * kMaxNbr * sizeof(int) : 0);
    t.mcnt = t.mnb + (mapr ? nm * kMaxNbr * sizeof(int) : 0);
    t.ell = (t.mcnt + (mapr ? (size_t)N : 0) + 3) / 4 * 4;
    t.err = t.ell + (aplm ? (size_t)E * sizeof(int) : 0);
    t.bytes = (t.err + (aplm ? (size_t)E * sizeof(int) : 0) + 15) / 16 * 16;
    return t;
}

// where the plane loop finds the column's angular-edge data: 0 the edge
// weights in global memory with the shared edge records (FP64); 1 the
// column's edge weights staged in LDS (FP32, four or five chunks per wave);
// 2 the column's edge table in LDS (FP32, up to three chunks per wave): for
// every direction and edge slot the upwind direction and the signed weight
constexpr int col_ang_mode(int real_bytes, int nch) {
    return real_bytes == 4 ? (nch <= 3 ? 2 : 1) : 0;
}

// one entry of the edge table: the edge term of a direction is w I_up (w
// zero for a slot past the direction's edges or an edge without motion)
struct alignas(8) AngEntry {
    int up;
    float w;
};

// angular-flux divergence from the edge table, in slot order with one
// rounding per term (the same value as angular_div_rec from the records)
__device__ __forceinline__ float ang_div_table(const AngEntry *__restrict__ t, int stride,
                                               const float *__restrict__ own, int n) {
    float div = 0.0f;
#pragma unroll
    for (int s = 0; s < kMaxNbr; ++s) {
        const AngEntry e = t[s * stride + n];
        div = ang_fma(e.w, own[e.up], div);
    }
    return div;
}

__device__ __forceinline__ void col_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// flag word of one direction of a column
constexpr unsigned kSxlP = 1u << 0, kSxlN = 1u << 1, kSxhP = 1u << 2, kSxhN = 1u << 3;
constexpr unsigned kSylP = 1u << 4, kSylN = 1u << 5, kSyhP = 1u << 6, kSyhN = 1u << 7;
constexpr unsigned kSzP = 1u << 8, kSzN = 1u << 9, kMsk = 1u << 10;
constexpr int kGhostShift = 16;   // bits 16..23: neighbour slot k (x-2, x-1, x+1, x+2,
                                  // y-2, y-1, y+1, y+2) reads zero (vacuum ghost)

__device__ __forceinline__ unsigned sign_bits(int s, unsigned pos, unsigned neg) {
    return s > 0 ? pos : (s < 0 ? neg : 0u);
}

// upwind values of the lower face (between the cells of v[1] and v[2]) and
// the upper face (v[2], v[3]) of the cell v[2]: from the left cell its
// value plus half its van Leer slope, from the right cell its value minus
// half of it; written exactly as the general kernel's axis_div forms them
template <typename Real>
__device__ __forceinline__ void axis_faces(const Real (&v)[5], bool plm, unsigned lo_p,
                                           unsigned lo_n, unsigned hi_p, unsigned hi_n,
                                           Real &ulo, Real &uhi) {
    Real hlm = Real(0), hl0 = Real(0), hlp = Real(0);
    if (plm) {
        hlm = half_slope(v[0], v[1], v[2]);
        hl0 = half_slope(v[1], v[2], v[3]);
        hlp = half_slope(v[2], v[3], v[4]);
    }
    ulo = lo_p ? v[1] + hlm : (lo_n ? v[2] - hl0 : Real(0));
    uhi = hi_p ? v[2] + hl0 : (hi_n ? v[3] - hlp : Real(0));
}

// the same face values with one select a face: a direction without motion
// across a face has a zero coefficient there (C = dA n^a n_0 with n^a = 0),
// so its value, the other upwind choice here, contributes a zero flux all the
// same (up to the sign of zero)
template <typename Real>
__device__ __forceinline__ void axis_faces2(const Real (&v)[5], bool plm, unsigned lo_p,
                                            unsigned hi_p, Real &ulo, Real &uhi) {
    Real hlm = Real(0), hl0 = Real(0), hlp = Real(0);
    if (plm) {
        hlm = half_slope(v[0], v[1], v[2]);
        hl0 = half_slope(v[1], v[2], v[3]);
        hlp = half_slope(v[2], v[3], v[4]);
    }
    ulo = lo_p ? v[1] + hlm : v[2] - hl0;
    uhi = hi_p ? v[2] + hl0 : v[3] - hlp;
}

// VWLDS: the column's angular-edge data staged in LDS (FP32; col_ang_mode
// says which form).  SPL: waves per
// column; with SPL = 2 the column's direction chunks split over two waves
// (NCH each) of the same workgroup, which share the cell's row through LDS
// and add their partial FP64 angle sums there (half 0's first); both then
// solve the same quartic
// One stage of the two-stage integrator (STG): Q* = gI q I + gB q Ib - beta
// dt (flux terms), the coupling starts from gT T + gTb Tb and runs over
// beta dt, and the bookkeeping and the masked-energy ledger carry the weight
// wS (the general kernel's stage, term for term).
template <typename Real>
struct ColStage {
    const Real *Ib;
    const double *Tb;
    double gI, gB, beta, gT, gTb, wS;
};

template <typename Real, int NCH, bool VWLDS, int SPL, int ANG, bool SUB, bool STG, bool TAU>
__global__ __launch_bounds__(kColBlock) __attribute__((amdgpu_waves_per_eu(col_waves<Real, NCH, TAU>()))) void k_column(
    DevGrid G, ColumnInfo CI, const Real *__restrict__ Iin, Real *__restrict__ Iout,
    double *__restrict__ T, const double *__restrict__ rho, const double *__restrict__ uvec,
    const double *__restrict__ kap_a, const double *__restrict__ kap_s, double dt_step,
    double *__restrict__ dT0, double *__restrict__ partials, int *__restrict__ nr_partial,
    Real *__restrict__ Istar, ColStage<Real> st) {
    const double dt = STG ? st.beta * dt_step : dt_step;   // this stage's time step
    const int lane = threadIdx.x % kWave;
    // wave-uniform (scalar registers): the column and every row address
    // derived from it
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int wc = wave / SPL, hh = wave % SPL;   // column slot, half
    const int lbase = lane + kWave * NCH * hh;   // this wave's first direction
    const int N = G.nang;
    const int E = G.nedge;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    // the direction tables every plane reads -- unit vectors, solid angles,
    // angular-edge records -- staged once per workgroup, so the plane loop
    // issues no global load behind the neighbour-row prefetch (vector-memory
    // counters retire in order: a later load's wait would also wait for it)
    // ANG: angular face values, 0 donor cell, 1 PLM (latitude-longitude
    // grids), 2 MAPR (geodesic); PLM and MAPR gather with the edge records
    // and weights, not the edge table
    constexpr int AM = VWLDS ? (ANG != 0 ? 1 : col_ang_mode(4, NCH)) : 0;
    constexpr int NHS = NCH * SPL * kWave;   // unit-vector component stride
    constexpr bool kMCM = sizeof(Real) == 4;  // MAPR tables component-major
    const ColTab TB = col_tab(N, E, NHS, sizeof(Real), AM != 2, ANG == 2, ANG == 1);
    double *s_nhat = reinterpret_cast<double *>(s_dyn + TB.nhat);   // [3][NHS]
    double *s_dom = reinterpret_cast<double *>(s_dyn + TB.dom);     // [N]
    int *s_adj = reinterpret_cast<int *>(s_dyn + TB.adj);           // [N][6] (not with AM 2)
    Real *s_minv = reinterpret_cast<Real *>(s_dyn + TB.minv);       // MAPR
    Real *s_md = reinterpret_cast<Real *>(s_dyn + TB.md);
    int *s_mnb = reinterpret_cast<int *>(s_dyn + TB.mnb);
    int8_t *s_mcnt = reinterpret_cast<int8_t *>(s_dyn + TB.mcnt);
    int *s_ell = reinterpret_cast<int *>(s_dyn + TB.ell);           // angular PLM
    int *s_err = reinterpret_cast<int *>(s_dyn + TB.err);
    // per column: the cell's row, double-buffered [2][own_stride], then the
    // column's edge weights [2E] (AM 1) or edge table [6][own_stride] (AM 2),
    // then with MAPR the row's gradients [own_stride][2]
    Real *s_row = reinterpret_cast<Real *>(s_dyn + CI.tab_bytes) + (size_t)wc * CI.col_lds;
    Real *s_vw = s_row + 2 * CI.own_stride;
    AngEntry *s_ang = reinterpret_cast<AngEntry *>(s_vw);
    Real *s_grad = s_vw + (AM == 1 ? 2 * E : (AM == 2 ? 2 * kMaxNbr * CI.own_stride : 0));
    __shared__ double s_x[kColWaves][8];   // partial angle sums of each wave (SPL = 2)
    __shared__ double s_v[kColWaves][8];   // the velocity substitute's partial sums (SPL = 2)
    // optical-depth-aware flux, per wave and plane: (u^0^, u^a^, alpha_E) of
    // the cell and its six face neighbours (x-, x+, y-, y+, z-, z+) and the
    // interpolating factor f of the six faces (x-, x+, y-, y+, z-, z+)
    __shared__ double s_tau[TAU ? kColWaves : 1][7][5];
    __shared__ double s_ftau[TAU ? kColWaves : 1][6];
    if constexpr (AM != 2)
        for (int k = threadIdx.x; k < N * kMaxNbr; k += kColBlock) s_adj[k] = edge_record(G, k);
    // unit vectors by component, so a wave's reads of one component are
    // consecutive in LDS
    for (int k = threadIdx.x; k < 3 * N; k += kColBlock) s_nhat[(k % 3) * NHS + k / 3] = G.nhat[k];
    if constexpr (ANG == 1) {
        for (int k = threadIdx.x; k < E; k += kColBlock) {
            s_ell[k] = G.edge_ll[k];
            s_err[k] = G.edge_rr[k];
        }
    }
    if constexpr (ANG == 2) {
        const Real *minv = static_cast<const Real *>(G.mapr_inv);
        const Real *md = static_cast<const Real *>(G.mapr_d);
        for (int k = threadIdx.x; k < N * kMaxNbr * 4; k += kColBlock)
            s_minv[kMCM ? (k % (kMaxNbr * 4)) * NHS + k / (kMaxNbr * 4) : k] = minv[k];
        for (int k = threadIdx.x; k < E * 4; k += kColBlock) s_md[k] = md[k];
        for (int k = threadIdx.x; k < N * kMaxNbr; k += kColBlock)
            s_mnb[kMCM ? (k % kMaxNbr) * NHS + k / kMaxNbr : k] = G.mapr_nb[k];
        for (int k = threadIdx.x; k < N; k += kColBlock) s_mcnt[k] = G.mapr_cnt[k];
    }
    for (int k = threadIdx.x; k < N; k += kColBlock) s_dom[k] = G.domega[k];
    __shared__ double s_E0[kColWaves][16];   // E0 of each wave's column

    // XCD-aware logical block: the hardware hands block b to XCD b % 8
    const int per = gridDim.x / 8;
    const int logical = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    // a workgroup's four waves take four neighbouring columns along axis 0;
    // workgroups run through bands of kColBand rows along axis 1, quad by
    // quad with the rows of the band fastest, so the axis-1 neighbours (and,
    // a band's height later, the axis-0 neighbours) of a column march at
    // the same time and its neighbour rows are read from L2
    const long long pcells = (long long)G.n0 * G.n1;
    constexpr int kCols = kColWaves / SPL;   // columns per workgroup
    const int nq = (G.n0 + kCols - 1) / kCols;
    const long long per_seg = (long long)nq * G.n1;
    const int seg = (int)(logical / per_seg);
    const int r = (int)(logical % per_seg);
    const int nband = (G.n1 + kColBand - 1) / kColBand;
    const int band = min(r / (nq * kColBand), nband - 1);
    const int h = min(kColBand, G.n1 - band * kColBand);   // rows of this band
    const int t = r - band * nq * kColBand;
    int i = (t / h) * kCols + wc, j = band * kColBand + t % h, z0 = 0, z1 = 0;
    // `active`: the wave marches (with SPL = 2 every wave of a workgroup with
    // work does, since the halves meet at barriers every plane; a column past
    // the grid's edge then marches the edge column and writes nothing);
    // `writes`: its results are stored
    const bool wg_on = seg < CI.nseg;
    const bool col_ok = i < G.n0;
    const bool active = SPL == 1 ? (wg_on && col_ok) : wg_on;
    const bool writes = wg_on && col_ok;
    if (active) {
        z0 = seg * CI.seglen;
        z1 = min(G.n2, z0 + CI.seglen);
        i = min(i, G.n0 - 1);
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
    const Real *vw = static_cast<const Real *>(G.vw);
    const Real ivol = static_cast<const Real *>(G.invV)[x.gc];
    const double volD = G.volD[x.gc];
    const double n0 = G.n0u[x.gc];
    if (lane < 16) s_E0[wave][lane] = G.E0[16 * x.gc + lane];
    const bool plm = G.recon == RT_RECON_PLM;
    const Real dtR = Real(dt);

    // ------------------------------------------------ column geometry, once
    const int fxl = face_geo(G, 0, i, x), fxh = face_geo(G, 0, i + 1, x);
    const int fyl = face_geo(G, 1, j, x), fyh = face_geo(G, 1, j + 1, x);
    const int fz = face_geo(G, 2, 0, x);   // every axis-2 face of the column
    // neighbour columns along axes 0 and 1 and the faces beyond which a
    // vacuum ghost sits (-1: the neighbour is an active or periodic cell)
    int ncol[8], gface[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int a = k / 4;
        const int o = (k % 4) < 2 ? (k % 4) - 2 : (k % 4) - 1;
        const int coord = a == 0 ? i : j;
        const int len = a == 0 ? G.n0 : G.n1;
        int idx = coord + o;
        gface[k] = -1;
        if (idx < 0 || idx >= len) {
            const int side = idx < 0 ? 0 : 1;
            if (G.bc[a][side] == RT_BC_PERIODIC) {
                idx = ((idx % len) + len) % len;
            } else {
                gface[k] = face_geo(G, a, side ? len : 0, x);
                idx = side ? len - 1 : 0;
            }
        }
        ncol[k] = a == 0 ? j * G.n0 + idx : idx * G.n0 + i;
    }
    // whether a vacuum ghost borders the column along axis 0 or 1 (wave-
    // uniform: most columns have none and skip the per-direction zeroing)
    const bool ghost_x = gface[0] >= 0 || gface[1] >= 0 || gface[2] >= 0 || gface[3] >= 0;
    const bool ghost_y = gface[4] >= 0 || gface[5] >= 0 || gface[6] >= 0 || gface[7] >= 0;
    Real gq[NCH], cxl[NCH], cxh[NCH], cyl[NCH], cyh[NCH], czz[NCH];
    unsigned fl[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int n = lbase + kWave * ch;
        const int m = n < N ? n : 0;
        const Real *C0 = static_cast<const Real *>(G.C[0]);
        const Real *C1 = static_cast<const Real *>(G.C[1]);
        const Real *C2 = static_cast<const Real *>(G.C[2]);
        gq[ch] = q[(size_t)x.gc * N + m];
        cxl[ch] = C0[(size_t)fxl * N + m];
        cxh[ch] = C0[(size_t)fxh * N + m];
        cyl[ch] = C1[(size_t)fyl * N + m];
        cyh[ch] = C1[(size_t)fyh * N + m];
        czz[ch] = C2[(size_t)fz * N + m];
        unsigned f = sign_bits(G.sgn[0][(size_t)fxl * N + m], kSxlP, kSxlN) |
                     sign_bits(G.sgn[0][(size_t)fxh * N + m], kSxhP, kSxhN) |
                     sign_bits(G.sgn[1][(size_t)fyl * N + m], kSylP, kSylN) |
                     sign_bits(G.sgn[1][(size_t)fyh * N + m], kSyhP, kSyhN) |
                     sign_bits(G.sgn[2][(size_t)fz * N + m], kSzP, kSzN);
        if (G.mask[(size_t)x.gc * N + m]) f |= kMsk;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (gface[k] < 0) continue;
            // ghost beyond a lower (slots 0, 1) or upper face: the edge cell
            // for directions leaving through it, zero for directions entering
            const int s = G.sgn[k / 4][(size_t)gface[k] * N + m];
            const bool out = (k % 4) < 2 ? (s < 0) : (s > 0);
            if (!out) f |= 1u << (kGhostShift + k);
        }
        fl[ch] = f;
    }
    if (AM == 1 && active && hh == 0) {
        const Real *row = vw + (size_t)x.gc * E * 2;
        for (int k = lane; k < 2 * E; k += kWave) s_vw[k] = row[k];
    }
    if constexpr (AM == 2) {
        // each wave the entries of its own directions: the upwind side of an
        // edge follows the sign of its angular motion v, the weight is +-w
        // (+ when the direction is the edge's lower one)
        if (active) {
            const Real *row = vw + (size_t)x.gc * E * 2;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lbase + kWave * ch;
                if (n >= N) continue;
                for (int sl = 0; sl < kMaxNbr; ++sl) {
                    AngEntry en{n, 0.0f};
                    const int e = G.has_edges ? G.adj_e[n * kMaxNbr + sl] : -1;
                    if (e >= 0) {
                        const float vv = row[2 * e], ww = row[2 * e + 1];
                        const float sw = G.adj_s[n * kMaxNbr + sl] > 0 ? ww : -ww;
                        if (vv > 0.0f) en = AngEntry{G.edge_lo[e], sw};
                        else if (vv < 0.0f) en = AngEntry{G.edge_hi[e], sw};
                    }
                    s_ang[sl * CI.own_stride + n] = en;
                }
            }
        }
    }
    const Real *vwrow = AM == 1 ? s_vw : vw + (size_t)x.gc * E * 2;
    __syncthreads();   // direction tables, s_vw

    double lum_acc = 0.0, me_acc = 0.0;
    int nr_acc = 0;
    if (active) {
        // plane pz of column `col` for the lane's directions as stored (the
        // wrapped or edge plane), and the axis-2 boundary condition to apply
        // to it: vacuum ghosts keep the edge cell only for directions leaving
        // through that face (`need` bit; 0: kept as read).  Applied where the
        // plane enters the queue, so a prefetch is not waited for at issue.
        auto load_raw = [&](int pz, int col, Real (&dst)[NCH]) -> unsigned {
            long long zz = pz;
            unsigned need = 0;
            if (pz < 0 || pz >= G.n2) {
                const int side = pz < 0 ? 0 : 1;
                if (G.bc[2][side] == RT_BC_PERIODIC) {
                    zz = ((pz % G.n2) + G.n2) % G.n2;
                } else {
                    need = side ? kSzP : kSzN;
                    zz = side ? G.n2 - 1 : 0;
                }
            }
            const Real *src = Iin + (zz * pcells + col) * N;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lbase + kWave * ch;
                dst[ch] = src[ch < NCH - 1 ? n : min(n, N - 1)];
            }
            return need;
        };
        auto apply_bc = [&](unsigned need, Real (&v)[NCH]) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                v[ch] = (need == 0 || (fl[ch] & need)) ? v[ch] : Real(0);
        };
        auto load_row = [&](int pz, int col, Real (&dst)[NCH]) {
            apply_bc(load_raw(pz, col, dst), dst);
        };
        // the four neighbour rows of axis a (0 or 1) at plane pz
        auto load_axis = [&](int pz, int a, Real (&dst)[4][NCH]) {
            const Real *base = Iin + (long long)pz * pcells * N;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * a + kk;
                const bool need = plm || kk == 1 || kk == 2;
                const Real *src = base + (long long)ncol[k] * N;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lbase + kWave * ch;
                    const Real v = need ? src[ch < NCH - 1 ? n : min(n, N - 1)] : Real(0);
                    dst[kk][ch] = (fl[ch] & (1u << (kGhostShift + k))) ? Real(0) : v;
                }
            }
        };
        // FP32: the next plane's eight neighbour rows are prefetched into
        // registers, as loaded (the vacuum-ghost zeros applied where they are
        // used), where that costs no resident wave: up to three chunks stay
        // at three waves per SIMD, five and six at two (at four the rows
        // would take the third wave away).  Faster than moving them into LDS
        // by global_load_lds (128 x 64 x 128 x 162: 3.17 against 3.27 ms),
        // which at six chunks would also leave one workgroup per CU.
        constexpr bool RPF = sizeof(Real) == 4 && NCH != 4;
        auto load_rows_raw = [&](int pz, Real (&dst)[8][NCH]) {
            const Real *base = Iin + (long long)pz * pcells * N;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const bool need = plm || (k % 4 == 1) || (k % 4 == 2);
                const Real *src = base + (long long)ncol[k] * N;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lbase + kWave * ch;
                    dst[k][ch] = need ? src[ch < NCH - 1 ? n : min(n, N - 1)] : Real(0);
                }
            }
        };
        const int mycol = (int)x.c;
        Real pnb[RPF ? 8 : 1][NCH];
        if constexpr (RPF) load_rows_raw(z0, pnb);
        // planes z-1 .. z+2 of the column; the lower axis-2 face flux of the
        // segment's first plane is formed here (it also needs plane z0-2)
        Real qz[4][NCH];
#pragma unroll
        for (int p = 0; p < 4; ++p) load_row(z0 - 1 + p, mycol, qz[p]);
        // optical-depth-aware flux (Sec. 2): lane k < 7 loads the fluid of the
        // cell (k = 0) or its face neighbour k at plane pz (a ghost carries the
        // cell's own fluid, a periodic neighbour wraps); tau_plane forms their
        // u^0^ and alpha_E and the faces' f = -expm1(-tau^2), tau = tau_coeff
        // alpha_E dt / u^0^ from the two cells' averages (the full step's dt)
        const bool zper = G.bc[2][0] == RT_BC_PERIODIC;
        auto tau_load = [&](int pz, double (&tf)[6]) {
            long long zz = pz;
            int col = mycol;
            if (lane == 1) col = ncol[1];
            if (lane == 2) col = ncol[2];
            if (lane == 3) col = ncol[5];
            if (lane == 4) col = ncol[6];
            if (lane == 5) zz = pz - 1 < 0 ? (zper ? G.n2 - 1 : pz) : pz - 1;
            if (lane == 6) zz = pz + 1 >= G.n2 ? (zper ? 0 : pz) : pz + 1;
            const long long cc = zz * pcells + col;
            tf[0] = uvec[3 * cc];
            tf[1] = uvec[3 * cc + 1];
            tf[2] = uvec[3 * cc + 2];
            tf[3] = rho[cc];
            tf[4] = kap_a[cc];
            tf[5] = kap_s[cc];
        };
        auto tau_plane = [&](const double (&tf)[6]) {
            if (lane < 7) {
                s_tau[wave][lane][0] = sqrt(1.0 + tf[0] * tf[0] + tf[1] * tf[1] + tf[2] * tf[2]);
                s_tau[wave][lane][1] = tf[0];
                s_tau[wave][lane][2] = tf[1];
                s_tau[wave][lane][3] = tf[2];
                s_tau[wave][lane][4] = (tf[4] + tf[5]) * tf[3];
            }
            col_wave_sync();
            if (lane < 6) {
                // face lane: lower faces (even) between neighbour 1 + lane and
                // the cell, upper faces (odd) between the cell and 1 + lane
                const int a = (lane & 1) ? 0 : 1 + lane, b = (lane & 1) ? 1 + lane : 0;
                const double t = G.tau_coeff * (0.5 * (s_tau[wave][a][4] + s_tau[wave][b][4])) *
                                 dt_step / (0.5 * (s_tau[wave][a][0] + s_tau[wave][b][0]));
                s_ftau[wave][lane] = -expm1(-t * t);
            }
            col_wave_sync();
        };
        // fluid-frame n^0bar of direction n in cell k of the block above
        auto tau_nb = [&](int k, int n) -> double {
            return s_tau[wave][k][0] - (s_tau[wave][k][1] * s_nhat[n] + s_tau[wave][k][2] * s_nhat[NHS + n] +
                                        s_tau[wave][k][3] * s_nhat[2 * NHS + n]);
        };
        if constexpr (TAU) {
            double tf[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (lane < 7) tau_load(z0, tf);
            tau_plane(tf);
        }
        Real Fz[NCH];
        {
            Real below[NCH];
            load_row(z0 - 2, mycol, below);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const Real v[5] = {Real(0), below[ch], qz[0][ch], qz[1][ch], qz[2][ch]};
                Real ulo, uhi;
                axis_faces(v, plm, 0u, 0u, fl[ch] & kSzP, fl[ch] & kSzN, ulo, uhi);
                (void)ulo;
                if constexpr (TAU) {
                    // the segment's lower face: between z0-1 (below) and z0
                    const int m = min(lbase + kWave * ch, N - 1);
                    double fL, fR;
                    tau_face(s_ftau[wave][4], tau_nb(5, m), tau_nb(0, m), fL, fR);
                    uhi *= Real((fl[ch] & kSzP) ? fL : fR);
                }
                Fz[ch] = czz[ch] * uhi;
            }
        }
        const bool lum_col = (G.lum_axis == 0 && i == (G.lum_side ? G.n0 - 1 : 0)) ||
                             (G.lum_axis == 1 && j == (G.lum_side ? G.n1 - 1 : 0));

        for (int z = z0; z < z1; ++z) {
            const long long c = (long long)z * pcells + x.c;
            const bool more = z + 1 < z1;
            // this plane's bookkeeping row (lanes 0..3) and beam flag, read
            // before the prefetches are issued so their waits do not include them
            double dpre = 0.0;
            if (dT0 && lane < 4) dpre = dT0[4 * c + lane];
            const int bflag = G.beam != nullptr ? (int)G.beam[c] : 0;
            // the column's next plane while this one is computed
            Real qn[NCH];
            unsigned qneed = 0;
            // the plane's fluid for the optical-depth-aware flux, before the
            // prefetch as well
            double tfl[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if constexpr (TAU) {
                if (lane < 7) tau_load(z, tfl);
            }
            if (more) qneed = load_raw(z + 3, mycol, qn);
            // the cell's row into LDS for the angular gather (double-buffered:
            // the other buffer's readers finished during the previous plane)
            Real *s_own = s_row + ((z - z0) & 1) * CI.own_stride;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lbase + kWave * ch;
                if (n < N) s_own[n] = qz[1][ch];
            }
            if constexpr (SPL == 1)
                col_wave_sync();
            else
                __syncthreads();
            if constexpr (ANG == 2) {
                // MAPR: every direction's gradient from the cell's row, then
                // shared with the gather through LDS (the previous plane's
                // readers passed this plane's row barrier, or, one wave per
                // column, read in program order)
                if (G.has_edges) {
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        const int n = lbase + kWave * ch;
                        if (n >= N) continue;
                        Real gx, gy;
                        if constexpr (kMCM)
                            mapr_gradient_t((int)s_mcnt[n], s_mnb + n, NHS, s_minv + n, NHS, s_own,
                                            n, gx, gy);
                        else
                            mapr_gradient_t((int)s_mcnt[n], s_mnb + n * kMaxNbr, 1,
                                            s_minv + (size_t)n * kMaxNbr * 4, 1, s_own, n, gx, gy);
                        s_grad[2 * n] = gx;
                        s_grad[2 * n + 1] = gy;
                    }
                    if constexpr (SPL == 1)
                        col_wave_sync();
                    else
                        __syncthreads();
                }
            }
            // 1/n^0bar of each direction in the cell (it borders all six faces)
            double tinc[TAU ? NCH : 1];
            if constexpr (TAU) {
                tau_plane(tfl);
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) tinc[ch] = rcp64(tau_nb(0, min(lbase + kWave * ch, N - 1)));
            }
            const bool lum_here = lum_col || (G.lum_axis == 2 && z == (G.lum_side ? G.n2 - 1 : 0));
            // ------------------------------------------------------ transport
            // axis by axis (one axis's neighbour rows live at a time)
            Real dq[NCH];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) dq[ch] = Real(0);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                Real nb[4][NCH];
                if constexpr (RPF) {
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch) nb[kk][ch] = pnb[4 * a + kk][ch];
                    if (a == 0 ? ghost_x : ghost_y) {
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch) {
                            // the flag tests are formed here, not kept as
                            // lane masks across the march
                            unsigned f = fl[ch];
                            asm volatile("" : "+v"(f));
#pragma unroll
                            for (int kk = 0; kk < 4; ++kk)
                                if (f & (1u << (kGhostShift + 4 * a + kk))) nb[kk][ch] = Real(0);
                        }
                    }
                } else {
                    load_axis(z, a, nb);
                }
                const unsigned lp = a ? kSylP : kSxlP, hp = a ? kSyhP : kSxhP;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lbase + kWave * ch;
                    const unsigned f = fl[ch];
                    const Real v[5] = {nb[0][ch], nb[1][ch], qz[1][ch], nb[2][ch], nb[3][ch]};
                    Real ulo, uhi;
                    axis_faces2(v, plm, f & lp, f & hp, ulo, uhi);
                    if constexpr (TAU) {
                        const int m = min(n, N - 1);
                        const double ilo = rcp64(tau_nb(1 + 2 * a, m));
                        const double ihi = rcp64(tau_nb(2 + 2 * a, m));
                        double fL, fR;
                        tau_face_inv(s_ftau[wave][2 * a], ilo, tinc[ch], fL, fR);
                        ulo *= Real((f & lp) ? fL : fR);
                        tau_face_inv(s_ftau[wave][2 * a + 1], tinc[ch], ihi, fL, fR);
                        uhi *= Real((f & hp) ? fL : fR);
                    }
                    const Real Flo = (a ? cyl[ch] : cxl[ch]) * ulo;
                    const Real Fhi = (a ? cyh[ch] : cxh[ch]) * uhi;
                    if (lum_here && G.lum_axis == a && n < N)
                        lum_acc += G.lum_side ? -s_dom[n] * (double)Fhi : s_dom[n] * (double)Flo;
                    dq[ch] += Fhi - Flo;
                }
            }
            if constexpr (RPF) {
                if (more) load_rows_raw(z + 1, pnb);
            }
            Real Is[NCH];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lbase + kWave * ch;
                const unsigned f = fl[ch];
                const Real Ic = qz[1][ch];
                {
                    const Real v[5] = {Real(0), qz[0][ch], Ic, qz[2][ch], qz[3][ch]};
                    Real ulo, uhi;
                    axis_faces2(v, plm, 0u, f & kSzP, ulo, uhi);
                    if constexpr (TAU) {
                        const int m = min(n, N - 1);
                        double fL, fR;
                        tau_face_inv(s_ftau[wave][5], tinc[ch], rcp64(tau_nb(6, m)), fL, fR);
                        uhi *= Real((f & kSzP) ? fL : fR);
                    }
                    (void)ulo;
                    const Real Flo = Fz[ch], Fhi = czz[ch] * uhi;
                    Fz[ch] = Fhi;
                    if (lum_here && G.lum_axis == 2 && n < N)
                        lum_acc += G.lum_side ? -s_dom[n] * (double)Fhi : s_dom[n] * (double)Flo;
                    dq[ch] += Fhi - Flo;
                }
                Is[ch] = Real(0);
                if (n >= N) continue;
                Real div = Real(0);
                if (G.has_edges) {
                    if constexpr (ANG == 2)
                        div = angular_div_mapr_t(s_md, s_adj, s_own, vwrow, s_grad, n);
                    else if constexpr (ANG == 1)
                        div = angular_div_plm_t(s_ell, s_err, s_adj, s_own, vwrow, n);
                    else if constexpr (AM == 2)
                        div = ang_div_table(s_ang, CI.own_stride, s_own, n);
                    else
                        div = angular_div_rec(s_adj, s_own, vwrow, n);
                }
                const Real qn_ = gq[ch];
                Real Qs = qn_ * Ic;
                if constexpr (STG) {
                    if (st.Ib) Qs = Real(st.gI) * Qs + Real(st.gB) * (qn_ * st.Ib[c * N + n]);
                }
                Qs = Qs - dtR * ivol * dq[ch] - quot(dtR * div, Real(s_dom[n]));
                if (f & kMsk) {
                    me_acc -= (STG ? st.wS : 1.0) * volD * s_dom[n] * (double)Qs;
                    continue;
                }
                Is[ch] = quot(Qs, qn_);
            }
            if (Istar && writes) {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lbase + kWave * ch;
                    if (n < N) Istar[c * N + n] = Is[ch];
                }
            }
            // ------------------------------------------------------ coupling
            double u1 = uvec[3 * c], u2 = uvec[3 * c + 1], u3 = uvec[3 * c + 2];
            double u0 = sqrt(fma(u1, u1, fma(u2, u2, fma(u3, u3, 1.0))));
            const double rh = rho[c];
            const double aa = kap_a[c] * rh, as = kap_s[c] * rh;
            const double tau = (aa + as) * dt;
            const double Tm = (STG && st.Tb) ? st.gT * T[c] + st.gTb * st.Tb[c] : T[c];
            if constexpr (SUB) {
                // radiation-dominated velocity substitute (Sec. 2.5): with the
                // gas velocity, E = sum I n0bar^2 dOm, R^00, R^0a and
                // sum n^a n0bar I dOm, then the substituted velocity couples
                double sv[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lbase + kWave * ch;
                    if (n >= N || (fl[ch] & kMsk)) continue;
                    const double nx = s_nhat[n], ny = s_nhat[NHS + n], nz = s_nhat[2 * NHS + n];
                    const double nb = u0 - fma(u1, nx, fma(u2, ny, u3 * nz));
                    const double Iw = (double)Is[ch] * s_dom[n];
                    const double Inb = Iw * nb;
                    sv[0] = fma(Inb, nb, sv[0]);
                    sv[1] += Iw;
                    sv[2] = fma(Iw, nx, sv[2]);
                    sv[3] = fma(Iw, ny, sv[3]);
                    sv[4] = fma(Iw, nz, sv[4]);
                    sv[5] = fma(Inb, nx, sv[5]);
                    sv[6] = fma(Inb, ny, sv[6]);
                    sv[7] = fma(Inb, nz, sv[7]);
                }
                wave_sum_quads(sv);
                if constexpr (SPL == 2) {
                    if (lane == 0) {
#pragma unroll
                        for (int k = 0; k < 8; ++k) s_v[wave][k] = sv[k];
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < 8; ++k) sv[k] = s_v[wc * SPL][k] + s_v[wc * SPL + 1][k];
                }
                velocity_substitute(sv, rh, Tm, aa, as, n0, dt, G.cv, G.kb, G.a_rad, u0, u1, u2, u3);
            }
            double nbv[NCH], rrv[NCH];
            double sf[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lbase + kWave * ch;
                const int m = n < N ? n : 0;
                const double nbr_ = u0 - fma(u1, s_nhat[m], fma(u2, s_nhat[NHS + m], u3 * s_nhat[2 * NHS + m]));
                const double nb2 = nbr_ * nbr_;
                const double rr = rcp64(nb2 * fma(nbr_, tau, n0));
                nbv[ch] = nbr_;
                rrv[ch] = rr;
                if (n >= N || (fl[ch] & kMsk)) continue;
                const double dom = s_dom[n];
                const double Iw = (double)Is[ch] * (nb2 * dom);
                sf[0] += Iw;
                sf[1] = fma(n0 * nb2 * rr, Iw, sf[1]);
                sf[2] = fma(dom, nbr_ * rr, sf[2]);
            }
            wave_sum_quads(sf);
            if constexpr (SPL == 2) {
                if (lane == 0) {
                    s_x[wave][0] = sf[0];
                    s_x[wave][1] = sf[1];
                    s_x[wave][2] = sf[2];
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 3; ++k) sf[k] = s_x[wc * SPL][k] + s_x[wc * SPL + 1][k];
            }
            const double Em = sf[0], A1 = sf[1], A2 = sf[2] * (dt / kFourPi);
            const double B4 = A2 * aa * G.a_rad;
            const double B1 = rh * G.cv * (1.0 - A2 * as);
            const double B0 = A1 - B1 * Tm - (1.0 - A2 * as) * Em;
            int bad = 0;
            const double Tp = quartic_root_fast(B4, B1, B0, bad, Tm);
            const double Ep = Em - rh * G.cv * (Tp - Tm);
            const double Tp2 = Tp * Tp;
            const double S = aa * G.a_rad * Tp2 * Tp2 + as * Ep;
            const double cS = S * (dt / kFourPi);
            double sm[4] = {0.0, 0.0, 0.0, 0.0};
            const bool beam_cell = bflag != 0;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lbase + kWave * ch;
                if (n >= N) continue;
                Real out = Real(0);
                if (!(fl[ch] & kMsk)) {
                    const double nbr_ = nbv[ch], rr = rrv[ch];
                    const double nbrr = nbr_ * rr;
                    const double dn = fma(nbr_, tau, n0);
                    const double I = (double)Is[ch];
                    const double Ip = fma(n0 * nbr_ * nbrr, I, cS * (nbrr * rr * dn));
                    const double dI = (Ip - I) * s_dom[n];
                    sm[0] += dI;
                    sm[1] = fma(dI, s_nhat[n], sm[1]);
                    sm[2] = fma(dI, s_nhat[NHS + n], sm[2]);
                    sm[3] = fma(dI, s_nhat[2 * NHS + n], sm[3]);
                    out = Real(Ip);
                }
                if (beam_cell && n == G.beam_angle) out = Real(G.beam_I);
                if (writes) Iout[c * N + n] = out;
            }
            if (lane == 0 && hh == 0 && writes) {
                T[c] = Tp;
                nr_acc += bad;
            }
            if (dT0) {
                wave_sum_quads(sm);
                if constexpr (SPL == 2) {
                    if (lane == 0) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) s_x[wave][4 + k] = sm[k];
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < 4; ++k) sm[k] = s_x[wc * SPL][4 + k] + s_x[wc * SPL + 1][4 + k];
                }
                if (lane < 4 && hh == 0 && writes) {
                    const double *E0 = s_E0[wave];
                    const int al = lane;
                    dT0[4 * c + al] = dpre - (STG ? st.wS : 1.0) * n0 * (E0[4 * al] * sm[0] + E0[4 * al + 1] * sm[1] +
                                                   E0[4 * al + 2] * sm[2] + E0[4 * al + 3] * sm[3]);
                }
            }
            if (more) {
                apply_bc(qneed, qn);
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    qz[0][ch] = qz[1][ch];
                    qz[1][ch] = qz[2][ch];
                    qz[2][ch] = qz[3][ch];
                    qz[3][ch] = qn[ch];
                }
            }
        }
    }
    // -------------------------------------------------------- block partials
    if (!writes) {
        lum_acc = 0.0;
        me_acc = 0.0;
        nr_acc = 0;
    }
    __shared__ double sh_l[kColWaves], sh_m[kColWaves];
    __shared__ int sh_n[kColWaves];
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
        for (int w = 0; w < kColWaves; ++w) {
            l += sh_l[w];
            m += sh_m[w];
            r += sh_n[w];
        }
        partials[2 * blockIdx.x] = l;
        partials[2 * blockIdx.x + 1] = m;
        nr_partial[blockIdx.x] = r;
    }
}

template <typename Real, int NCH, int SPL, int ANG, bool SUB, bool STG, bool TAU>
int launch_col(rt_grid *g, hipStream_t s, size_t lds, const void *Iin, void *Iout, double *T,
               const double *rho, const double *u, const double *ka, const double *ks, double dt,
               double *dT0, void *Istar, const Partials &P, const ColStage<Real> &st) {
    const ColumnInfo &CI = g->column;
    const auto kern = k_column<Real, NCH, sizeof(Real) == 4, SPL, ANG, SUB, STG, TAU>;
    if (ensure_dynamic_lds(reinterpret_cast<const void *>(kern), lds) != RT_OK) return RT_EDEVICE;
    hipLaunchKernelGGL(kern, dim3(CI.grid), dim3(kColBlock), lds, s, g->dg, CI,
                       static_cast<const Real *>(Iin), static_cast<Real *>(Iout), T, rho, u, ka, ks,
                       dt, dT0, P.sums, P.noroot, static_cast<Real *>(Istar), st);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

template <typename Real, int ANG, bool SUB, bool STG = false, bool TAU = false>
int launch_column_a(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                    const double *rho, const double *u, const double *ka, const double *ks,
                    double dt, double *dT0, void *Istar, const Partials &P,
                    const ColStage<Real> &st = ColStage<Real>{nullptr, nullptr, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0}) {
    const ColumnInfo &CI = g->column;
    const DevGrid &G = g->dg;
    const size_t lds = CI.tab_bytes + (size_t)(kColWaves / CI.split) * CI.col_lds * sizeof(Real);
    const int nch = (G.nang + kWave - 1) / kWave;
    // six chunks split over two waves (the only six-chunk variant)
    if (CI.split == 2) {
        if (nch != 6) return RT_EINVAL;
        return launch_col<Real, 3, 2, ANG, SUB, STG, TAU>(g, s, lds, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P, st);
    }
    if (CI.split != 1) return RT_EINVAL;
    switch (nch) {
        case 1: return launch_col<Real, 1, 1, ANG, SUB, STG, TAU>(g, s, lds, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P, st);
        case 2: return launch_col<Real, 2, 1, ANG, SUB, STG, TAU>(g, s, lds, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P, st);
        case 3: return launch_col<Real, 3, 1, ANG, SUB, STG, TAU>(g, s, lds, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P, st);
        case 4: return launch_col<Real, 4, 1, ANG, SUB, STG, TAU>(g, s, lds, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P, st);
        case 5: return launch_col<Real, 5, 1, ANG, SUB, STG, TAU>(g, s, lds, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P, st);
        default: return RT_EINVAL;
    }
}

template <typename Real>
int launch_column_t(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                    const double *rho, const double *u, const double *ka, const double *ks,
                    double dt, double *dT0, void *Istar, const Partials &P) {
    // PLM or MAPR, or the velocity substitute or the optical-depth-aware
    // flux with DC angular fluxes
    if (g->dg.tau_coeff > 0.0) {
        if (g->dg.ang_recon != 0 || g->dg.rad_velocity) return RT_EINVAL;
        return launch_column_a<Real, 0, false, false, true>(g, s, Iin, Iout, T, rho, u, ka, ks, dt,
                                                            dT0, Istar, P);
    }
    if (g->dg.rad_velocity) {
        if (g->dg.ang_recon != 0) return RT_EINVAL;
        return launch_column_a<Real, 0, true>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
    }
    if (g->dg.ang_recon == 2)
        return launch_column_a<Real, 2, false>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
    if (g->dg.ang_recon == 1)
        return launch_column_a<Real, 1, false>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
    if (g->dg.ang_recon != 0) return RT_EINVAL;
    return launch_column_a<Real, 0, false>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
}

}  // namespace

// Segments of the column march: enough workgroups to fill the chip several
// times over (about 32 wavefronts per CU), at least 4 planes per segment.
bool column_config(rt_grid *g, int seglen_hint) {
    ColumnInfo &CI = g->column;
    const DevGrid &G = g->dg;
    const long long cols = (long long)G.n0 * G.n1;
    long long seglen = seglen_hint > 0 ? seglen_hint
                                       : std::max<long long>(4, (G.n2 * cols + 8191) / 8192);
    seglen = std::min<long long>(seglen, G.n2);
    const long long nseg = (G.n2 + seglen - 1) / seglen;
    const long long nwork = cols * nseg;
    const int real = g->precision == RT_F32 ? 4 : 8;
    // up to six direction chunks in either precision (FP64 with five or six
    // spills a few registers and is still faster than the general kernel:
    // 256 x 128 x 256 x 362 Kerr-Schild 125 against 169 ms, 128 x 64 x 128 x
    // 162 5.9 against 7.5 ms)
    const int nch = (G.nang + kWave - 1) / kWave;
    if (nch > 6) return false;
    // six chunks: two waves per column (three chunks each, three resident
    // waves per SIMD instead of two)
    CI.split = nch == 6 ? 2 : 1;
    // one workgroup per quad (pair, when split) of columns along axis 0 (the
    // last of a row may be partly idle) per row and segment
    const int cols_wg = kColWaves / CI.split;
    const long long blocks = (long long)((G.n0 + cols_wg - 1) / cols_wg) * G.n1 * nseg;
    if (blocks >= (1LL << 30)) return false;
    CI.seglen = (int)seglen;
    CI.nseg = (int)nseg;
    CI.nwork = nwork;
    CI.grid = (int)((blocks + 7) / 8 * 8);
    CI.own_stride = (G.nang + 3) / 4 * 4;
    // as the launcher instantiates: direction chunks per wave, where the
    // plane loop finds the angular-edge data, the MAPR tables
    const bool mapr = G.ang_recon == 2, aplm = G.ang_recon == 1;
    const int nchw = CI.split == 2 ? 3 : nch;
    const int am = real == 4 ? (G.ang_recon != 0 ? 1 : col_ang_mode(real, nchw)) : 0;
    CI.tab_bytes =
        col_tab(G.nang, G.nedge, nchw * CI.split * kWave, real, am != 2, mapr, aplm).bytes;
    // per column: the cell's row twice, then the FP32 edge weights or the
    // edge table (two words an entry), then the MAPR gradients
    CI.col_lds = 2 * CI.own_stride + (am == 1 ? 2 * G.nedge : (am == 2 ? 2 * kMaxNbr * CI.own_stride : 0)) +
                 (mapr ? 2 * CI.own_stride : 0);
    // within the default dynamic LDS limit; with MAPR's tables up to half a
    // CU's LDS (two workgroups per CU), beyond which the general kernel runs
    const size_t lds = CI.tab_bytes + (size_t)cols_wg * CI.col_lds * real;
    return lds <= (mapr ? 80 : 64) * 1024;
}

// The two-stage (Heun) step on the column path: stage 1 from (I, T) into
// the stage buffers, stage 2 from them back into (Iout, T) with the blend of
// both states; the luminosity takes half of each stage.
template <typename Real>
int column_rk2_t(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                 const double *rho, const double *u, const double *ka, const double *ks,
                 double dt, double *dT0, double *lum, const Partials &P) {
    const size_t ncell = (size_t)g->dg.n0 * g->dg.n1 * g->dg.n2;
    if (hipMemcpyAsync(g->stage_T, T, ncell * sizeof(double), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return RT_EDEVICE;
    const ColStage<Real> s1{nullptr, nullptr, 1.0, 0.0, 1.0, 1.0, 0.0, 0.5};
    const bool tau = g->dg.tau_coeff > 0.0;
    int rc = tau ? launch_column_a<Real, 0, false, true, true>(g, s, Iin, g->stage_I, g->stage_T, rho,
                                                              u, ka, ks, dt, dT0, nullptr, P, s1)
                 : launch_column_a<Real, 0, false, true>(g, s, Iin, g->stage_I, g->stage_T, rho, u,
                                                         ka, ks, dt, dT0, nullptr, P, s1);
    if (rc == RT_OK) rc = launch_finalize(g, s, g->column.grid, 0.5 * dt, lum, P);
    if (rc != RT_OK) return rc;
    const ColStage<Real> s2{static_cast<const Real *>(Iin), g->stage_T, 0.5, 0.5, 0.5, 0.5, 0.5, 1.0};
    rc = tau ? launch_column_a<Real, 0, false, true, true>(g, s, g->stage_I, Iout, T, rho, u, ka, ks,
                                                          dt, dT0, nullptr, P, s2)
             : launch_column_a<Real, 0, false, true>(g, s, g->stage_I, Iout, T, rho, u, ka, ks, dt,
                                                     dT0, nullptr, P, s2);
    if (rc == RT_OK) rc = launch_finalize(g, s, g->column.grid, 0.5 * dt, lum, P);
    return rc;
}

int launch_column_rk2(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                      const double *rho, const double *u, const double *ka, const double *ks,
                      double dt, double *dT0, double *lum, const Partials &P) {
    if (g->dg.ang_recon != 0 || g->dg.rad_velocity) return RT_EINVAL;
    if (g->precision == RT_F32)
        return column_rk2_t<float>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
    return column_rk2_t<double>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
}

int launch_column(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                  const double *rho, const double *u, const double *ka, const double *ks,
                  double dt, double *dT0, void *Istar, const Partials &P) {
    if (g->precision == RT_F32)
        return launch_column_t<float>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
    return launch_column_t<double>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
}

}  // namespace rt
