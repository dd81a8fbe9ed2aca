// Hand-written adjoint of one radiation step (the reverse of k_step).
//
// Forward step s:  I* = L(I_s)  (transport, Sec. 2.3-2.4, 2.6),
//                  (I+, T+) = coupling(I*, T_s)  (Sec. 2.5),
//                  beam cells re-imposed,  J += w * dt * l(I_s).
// Given lamI = dJ/dI_{s+1}, lamT = dJ/dT_{s+1}, the adjoint step produces
// dJ/dI_s, dJ/dT_s and accumulates dJ/dkappa_a, dJ/dkappa_s, in two kernels:
//
//   k_adj_couple   (one wavefront per cell) recomputes I* and the forward
//                  coupling, then reverses it: the quartic root by the
//                  implicit-function theorem dT+/dB_k = -T+^k / P'(T+), the
//                  FP64 angle sums by their own adjoint sums.  Writes
//                  psi = (dJ/dI*) / (n^0 n_0) per cell-direction.
//   k_adj_transport (one lane per cell-direction; the tiled k_adj_march in
//                  its place for spatially uniform geometry, the column march
//                  k_adj_column for geometry independent of axis 2) gathers over the faces
//                  whose upwind value depends on the cell (radius 2): the
//                  direct term, the upwind PLM fluxes with the van Leer
//                  limiter's Jacobian on the branch the forward took, the
//                  angular upwind fluxes, and the luminosity seed.
#include <hip/hip_runtime.h>

#include "k_adj_common.h"

namespace rt {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kCellsPerBlock = 16;

// SW lanes per cell (16, 32 or 64; several cells per wavefront when SW < 64),
// lane l of a group handles directions l, l+SW, ... (NCH of them; every
// chunk but the last lies wholly below N, so only its indices need clamping).  RECOMP:
// recompute I* from I_n (else it is read from the forward step's output).
template <typename Real, int SW, int NCH, bool RECOMP>
__global__ __launch_bounds__(kBlock) void k_adj_couple(
    DevGrid G, const Real *__restrict__ Iin, const double *__restrict__ Tin,
    const double *__restrict__ rho, const double *__restrict__ uvec,
    const double *__restrict__ kap_a, const double *__restrict__ kap_s, double dt,
    const Real *__restrict__ lamI1, const double *__restrict__ lamT1, Real *__restrict__ psi,
    double *__restrict__ lamT0, double *__restrict__ gka, double *__restrict__ gks,
    const Real *__restrict__ Istar) {
    constexpr int kGroups = kBlock / SW;
    // unclamped chunk indices (constant offsets from the row base), except
    // in the FP64 16-lane variant, where they would cost its second wave
    constexpr bool kOpen = sizeof(Real) == 4 || SW == 64;
    const int lane = threadIdx.x % SW;
    const int grp = threadIdx.x / SW;
    const long long ncell = (long long)G.n0 * G.n1 * G.n2;
    const int N = G.nang;
    const Real *q = static_cast<const Real *>(G.q);
    const Real *invV = static_cast<const Real *>(G.invV);
    const Real dtR = Real(dt);
    double dummy_l = 0.0, dummy_m = 0.0;
    const bool uniform_geo = G.g0 == 1 && G.g1 == 1 && G.g2 == 1;
    // per-cell inputs of the stored-I* variant, prefetched one cell ahead
    // (the loads of the next cell are in flight while this one is computed)
    struct In {
        Real I[NCH], lp[NCH];
        double u1, u2, u3, rho, ka, ks, T, lT;
    };
    auto fetch = [&](long long c, In &v) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = (kOpen && ch < NCH - 1 ? lane + SW * ch : min(lane + SW * ch, N - 1));
            v.I[ch] = Istar[c * N + n];
            v.lp[ch] = lamI1[c * N + n];
        }
        v.u1 = uvec[3 * c];
        v.u2 = uvec[3 * c + 1];
        v.u3 = uvec[3 * c + 2];
        v.rho = rho[c];
        v.ka = kap_a[c];
        v.ks = kap_s[c];
        v.T = Tin[c];
        v.lT = lamT1[c];
    };
    // unit vectors and solid angles, staged per workgroup: the cell loop
    // then issues no global load of them behind the next cell's prefetch
    // (vector-memory counters retire in order, so such a load's wait would
    // also wait for the prefetch)
    extern __shared__ double s_tab[];
    double *s_nh = s_tab;          // [N][3]
    double *s_dom = s_tab + 3 * N; // [N]
    for (int k = threadIdx.x; k < 3 * N; k += kBlock) s_nh[k] = G.nhat[k];
    for (int k = threadIdx.x; k < N; k += kBlock) s_dom[k] = G.domega[k];
    __syncthreads();
    In cur{}, nxt{};
    {
        const long long c0 = (long long)blockIdx.x * kCellsPerBlock + grp;
        if constexpr (!RECOMP)
            if (c0 < ncell) fetch(c0, cur);
    }
    for (int cw = grp; cw < kCellsPerBlock; cw += kGroups) {
        const long long cc = (long long)blockIdx.x * kCellsPerBlock + cw;
        if (cc >= ncell) break;
        Cell x;
        if constexpr (RECOMP) {
            x = make_cell(G, cc);
        } else {
            // only the cell and its geometry index are needed (cell counts
            // stay far below 2^32, so 32-bit index arithmetic suffices)
            x.c = cc;
            x.gc = 0;
            if (!uniform_geo) {
                const unsigned cu = (unsigned)cc, n0 = (unsigned)G.n0, n1 = (unsigned)G.n1;
                const unsigned t = cu / n0;
                x.i = (int)(cu - t * n0);
                x.j = (int)(t % n1);
                x.k = (int)(t / n1);
                x.gc = ((G.g2 > 1 ? x.k : 0) * G.g1 + (G.g1 > 1 ? x.j : 0)) * G.g0 +
                       (G.g0 > 1 ? x.i : 0);
            }
        }
        // this cell's geometry rows, beam flag and gradient accumulators, read
        // before the next cell's prefetch is issued (so their waits do not
        // include it)
        // (the mask where the registers allow, q too with one cell per
        // wavefront; otherwise they are read where they are used)
        constexpr bool kMK = SW == 64 || NCH <= 6;
        constexpr bool kQ = SW == 64;
        unsigned char mk[NCH];
        Real qv[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int m = (kOpen && ch < NCH - 1 ? lane + SW * ch : min(lane + SW * ch, N - 1));
            if constexpr (kMK) mk[ch] = G.mask[(size_t)x.gc * N + m];
            if constexpr (kQ) qv[ch] = q[(size_t)x.gc * N + m];
        }
        const double n0 = G.n0u[x.gc];
        const int bm = G.beam != nullptr ? (int)G.beam[x.c] : 0;
        const double ga = gka ? gka[x.c] : 0.0, gs = gks ? gks[x.c] : 0.0;
        if constexpr (!RECOMP) {
            const long long cn = cc + kGroups;
            if (cw + kGroups < kCellsPerBlock && cn < ncell) fetch(cn, nxt);
        }
        if constexpr (RECOMP) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = (kOpen && ch < NCH - 1 ? lane + SW * ch : min(lane + SW * ch, N - 1));
                cur.I[ch] = transport_dir(G, Iin, x, n, dtR, invV[x.gc], dummy_l, dummy_m);
                cur.lp[ch] = lamI1[x.c * N + n];
            }
            cur.u1 = uvec[3 * x.c];
            cur.u2 = uvec[3 * x.c + 1];
            cur.u3 = uvec[3 * x.c + 2];
            cur.rho = rho[x.c];
            cur.ka = kap_a[x.c];
            cur.ks = kap_s[x.c];
            cur.T = Tin[x.c];
            cur.lT = lamT1[x.c];
        }
        Real Is[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) Is[ch] = ((kOpen && ch < NCH - 1) || lane + SW * ch < N) ? cur.I[ch] : Real(0);
        // forward coupling, recomputed.  Per direction: nb = n^0bar (fluid
        // frame), dn = n^0 + nb (alpha_a + alpha_s) dt, rr = 1/(nb^2 dn) and
        // from it idn = 1/dn, k = n^0/dn, 1/(nb dn) = nb rr; w = nb^2 dOmega.
        // Only nb and rr are kept per direction (registers); the rest is
        // re-formed where it is used.
        const double u1 = cur.u1, u2 = cur.u2, u3 = cur.u3;
        const double u0 = sqrt(fma(u1, u1, fma(u2, u2, fma(u3, u3, 1.0))));
        const double rh = cur.rho;
        const double aa = cur.ka * rh, as = cur.ks * rh;
        const double tau = (aa + as) * dt;
        double nbv[NCH], rrv[NCH];
        bool live[NCH];
        double sf[3] = {0.0, 0.0, 0.0};   // Em, A1, A2
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = lane + SW * ch;
            live[ch] = ((kOpen && ch < NCH - 1) || n < N) && !(kMK ? mk[ch] : G.mask[(size_t)x.gc * N + (n < N ? n : 0)]);
            const int m = live[ch] ? n : 0;
            const double nb = u0 - fma(u1, s_nh[3 * m], fma(u2, s_nh[3 * m + 1], u3 * s_nh[3 * m + 2]));
            const double nb2 = nb * nb;
            const double rr = rcp64(nb2 * fma(nb, tau, n0));
            nbv[ch] = nb;
            rrv[ch] = rr;
            const double dom = live[ch] ? s_dom[m] : 0.0;   // zero weight: masked or padding
            const double Iw = (double)Is[ch] * (nb2 * dom);
            sf[0] += Iw;
            sf[1] = fma(n0 * nb2 * rr, Iw, sf[1]);
            sf[2] = fma(dom, nb * rr, sf[2]);
        }
        group_sum_v<SW, 3>(sf);
        const double Em = sf[0], A1 = sf[1], A2 = sf[2] * (dt / kFourPi);
        const double Tm = cur.T;
        const double B4 = A2 * aa * G.a_rad;
        const double B1 = rh * G.cv * (1.0 - A2 * as);
        const double B0 = A1 - B1 * Tm - (1.0 - A2 * as) * Em;
        int bad = 0;
        const double Tp = quartic_root_fast(B4, B1, B0, bad, Tm);
        const double Ep = Em - rh * G.cv * (Tp - Tm);
        const double Tp3 = Tp * Tp * Tp;
        const double S = aa * G.a_rad * Tp3 * Tp + as * Ep;
        const double Pp = 4.0 * B4 * Tp3 + B1;
        // adjoint sums over directions: lS, X1, X2, X3
        const bool beam_cell = bm != 0;
        const double c4 = dt / kFourPi;
        double sr[4] = {0.0, 0.0, 0.0, 0.0};
        Real lpv[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = lane + SW * ch;
            const int m = live[ch] ? n : 0;
            const double nb = nbv[ch], rr = rrv[ch];
            const double nb2 = nb * nb;
            const double dn = fma(nb, tau, n0);
            const double idn = nb2 * rr;                          // 1/dn
            const double k = n0 * idn;                            // n^0/dn
            const double dom = live[ch] ? s_dom[m] : 0.0;
            const double I = (double)Is[ch];
            const double gdir = c4 * (nb * rr) * rr * dn;         // dt/(4 pi dn nb^3)
            const double nbdn = nb * idn;                         // nb/dn
            const bool use = live[ch] && !(beam_cell && n == G.beam_angle);
            const Real lpr = use ? cur.lp[ch] : Real(0);
            lpv[ch] = lpr;
            const double lp = (double)lpr;
            sr[0] = fma(lp, gdir, sr[0]);
            sr[1] = fma(lp * fma(I, k, S * gdir), nbdn, sr[1]);
            sr[2] = fma(nb2 * dom * I * k, nbdn, sr[2]);
            sr[3] = fma(dom * idn, idn, sr[3]);
        }
        group_sum_v<SW, 4>(sr);
        const double lS = sr[0], X1 = sr[1], X2 = sr[2], X3 = sr[3];
        // scalar reverse of S, Ep, the quartic and the B coefficients
        const double rcv = rh * G.cv;
        const double lEp = lS * as;
        const double lTp = cur.lT + lS * 4.0 * aa * G.a_rad * Tp3 - rcv * lEp;
        double lTm = rcv * lEp;
        double laa = lS * G.a_rad * Tp3 * Tp;
        double las = lS * Ep;
        const double iPp = rcp64(Pp);
        const double lB4 = -lTp * Tp3 * Tp * iPp;
        double lB1 = -lTp * Tp * iPp;
        const double lB0 = -lTp * iPp;
        const double lA1 = lB0;
        lB1 -= lB0 * Tm;
        lTm -= lB0 * B1;
        double lA2as = lB0 * Em;
        const double lEm = lEp - lB0 * (1.0 - A2 * as);
        lA2as -= rcv * lB1;
        double lA2 = lB4 * aa * G.a_rad;
        laa += lB4 * A2 * G.a_rad;
        lA2 += lA2as * as;
        las += lA2as * A2;
        const double ltau = -X1 - lA1 * X2 - lA2 * (dt / kFourPi) * X3;
        laa += ltau * dt;
        las += ltau * dt;
        // dJ/dI* per direction, divided by n^0 n_0
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = lane + SW * ch;
            if ((!kOpen || ch == NCH - 1) && n >= N) continue;
            Real out = Real(0);
            if (live[ch]) {
                const double nb = nbv[ch];
                const double nb2 = nb * nb;
                const double k = n0 * nb2 * rrv[ch];
                const double w = nb2 * s_dom[n];
                const double lstar = fma(k, (double)lpv[ch], fma(lA1, k, lEm) * w);
                out = Real(lstar * rcp64((double)(kQ ? qv[ch] : q[(size_t)x.gc * N + n])));
            }
            psi[x.c * N + n] = out;
        }
        if (lane == 0) {
            lamT0[x.c] = lTm;
            if (gka) gka[x.c] = ga + laa * rh;
            if (gks) gks[x.c] = gs + las * rh;
        }
        if constexpr (!RECOMP) cur = nxt;
    }
}

// Geometry-cell stride along axis a (0 if the geometry does not depend on a).
__device__ __forceinline__ int geo_stride(const DevGrid &G, int a) {
    if (a == 0) return G.g0 > 1 ? 1 : 0;
    if (a == 1) return G.g1 > 1 ? G.g0 : 0;
    return G.g2 > 1 ? G.g0 * G.g1 : 0;
}

template <typename Real, int NCH>
__global__ __launch_bounds__(kBlock) void k_adj_transport(DevGrid G, const Real *__restrict__ Iin,
                                                          const Real *__restrict__ psi, double dt,
                                                          double lum_weight,
                                                          Real *__restrict__ lamI0) {
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const long long ncell = (long long)G.n0 * G.n1 * G.n2;
    const int N = G.nang;
    const Real *q = static_cast<const Real *>(G.q);
    const Real *vw = static_cast<const Real *>(G.vw);
    const Real *invV = static_cast<const Real *>(G.invV);
    const Real dtR = Real(dt);
    const bool plm = G.recon == RT_RECON_PLM;

    for (int cw = wave; cw < kCellsPerBlock; cw += kWavesPerBlock) {
        const long long cc = (long long)blockIdx.x * kCellsPerBlock + cw;
        if (cc >= ncell) break;
        const Cell x = make_cell(G, cc);
        Real lam[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = lane + kWave * ch;
            const int m = n < N ? n : 0;
            // direct term: I*_c = I_c - (flux terms)
            lam[ch] = G.mask[(size_t)x.gc * N + m] ? Real(0) : psi[x.c * N + m] * q[(size_t)x.gc * N + m];
        }
        // axis by axis: the rows of the five cells and four faces the gather
        // touches are resolved once per cell (uniform across the wavefront)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int coord = axis_coord(x, a);
            const int len = axis_len(G, a);
            const long long stride = axis_stride(G, a);
            const int gstr = geo_stride(G, a);
            const bool periodic = G.bc[a][0] == RT_BC_PERIODIC;
            const Real *C = static_cast<const Real *>(G.C[a]);
            AxisRows<Real> R;
            axis_rows(G, Iin, x, a, R);
            // psi rows at offsets -2 .. +2 and their cells' 1/dV; outside a
            // non-periodic boundary the row is the edge cell's and 1/dV is
            // zero (psi only enters as psi / dV, so the product is zero)
            const Real *prow[5];
            Real iv[5];
#pragma unroll
            for (int o = -2; o <= 2; ++o) {
                int idx = coord + o;
                bool inside = idx >= 0 && idx < len;
                if (!inside && periodic) {
                    idx = ((idx % len) + len) % len;
                    inside = true;
                }
                const int ridx = inside ? idx : (idx < 0 ? 0 : len - 1);
                prow[o + 2] = psi + (x.c + (long long)(ridx - coord) * stride) * N;
                iv[o + 2] = inside ? invV[x.gc + (idx - coord) * gstr] : Real(0);
            }
            // faces at offsets fo = -1 .. 2 (face F between cells F-1 and F)
            const int8_t *Srow[4];
            const Real *Crow[4];
            bool fvalid[4], fon[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int fo = f - 1;
                const int Fraw = coord + fo;
                fvalid[f] = periodic || (Fraw >= 0 && Fraw <= len);
                const int F = periodic ? ((Fraw % len) + len) % len : Fraw;
                const int fg = face_geo(G, a, fvalid[f] ? F : 0, x);
                Srow[f] = G.sgn[a] + (size_t)fg * N;
                Crow[f] = C + (size_t)fg * N;
                // luminosity face (on a periodic axis the face between the last
                // and the first cell, where the forward step counts it)
                fon[f] = a == G.lum_axis && fvalid[f] &&
                         (periodic ? F == 0 : (G.lum_side == 1 ? F == len : F == 0));
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lane + kWave * ch;
                if (n >= N) continue;
                Real v[5], ps[5];
                v[2] = Iin[x.c * N + n];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    Real val = R.nb[k][n];
                    if (R.bs[k] != nullptr) {
                        const int sb = R.bs[k][n];
                        const bool out = k < 2 ? (sb < 0) : (sb > 0);
                        val = out ? val : Real(0);
                    }
                    v[k < 2 ? k : k + 1] = val;
                }
#pragma unroll
                for (int o = 0; o < 5; ++o) ps[o] = prow[o][n];
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    if (!fvalid[f]) continue;
                    const int fo = f - 1;
                    const int s = Srow[f][n];
                    if (s == 0) continue;
                    const int u = s > 0 ? fo - 1 : fo;       // upwind cell, relative to x
                    if (u < -1 || u > 1) continue;
                    if (!periodic && (coord + u < 0 || coord + u >= len)) continue;  // ghost upwind
                    // d V / d I_x (helpers shared with the column adjoint)
                    Real dh = Real(0);
                    if (plm) {
                        Real hx, hy;
                        half_slope_partials(v[u + 1], v[u + 2], v[u + 3], hx, hy);
                        dh = dh_at(u, hx, hy);
                    }
                    const Real d = face_weight(u == 0, s > 0, plm, dh);
                    // dJ/dF: the face is the upper face of cell fo-1 and the lower face of cell fo
                    Real lF = face_adjoint(dtR, ps[fo + 2], iv[fo + 2], ps[fo + 1], iv[fo + 1]);
                    if (fon[f]) lF += lum_seed<Real>(G, lum_weight, dt, n);
                    face_add(lam[ch], lF, Crow[f][n], d);
                }
            }
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = lane + kWave * ch;
            if (n >= N) continue;
            if (G.has_edges) {
                const Real a_n = psi[x.c * N + n] * Real(1.0 / G.domega[n]);
#pragma unroll
                for (int s = 0; s < kMaxNbr; ++s) {
                    const int e = G.adj_e[n * kMaxNbr + s];
                    if (e < 0) break;
                    const size_t vi = ((size_t)x.gc * G.nedge + e) * 2;
                    const Real vv = vw[vi], ww = vw[vi + 1];
                    const bool is_lo = G.adj_s[n * kMaxNbr + s] > 0;
                    const bool up = is_lo ? vv > Real(0) : vv < Real(0);
                    if (!up) continue;
                    const int p = is_lo ? G.edge_hi[e] : G.edge_lo[e];
                    edge_add(lam[ch], a_n, psi[x.c * N + p], Real(1.0 / G.domega[p]),
                             edge_weight(dtR, ww, is_lo));
                }
            }
            lamI0[x.c * N + n] = lam[ch];
        }
    }
}

template <typename Real>
int launch_adj_t(rt_grid *g, hipStream_t s, const void *Iin, const double *Tin,
                 const double *rho, const double *u, const double *ka, const double *ks,
                 double dt, double lum_weight, const void *lamI1, const double *lamT1,
                 void *lamI0, double *lamT0, void *work, double *gka, double *gks,
                 const void *Istar) {
    const DevGrid &G = g->dg;
    const long long ncell = (long long)G.n0 * G.n1 * G.n2;
    const int nblk = (int)((ncell + kCellsPerBlock - 1) / kCellsPerBlock);
    const int nch = (G.nang + kWave - 1) / kWave;
    const Real *in = static_cast<const Real *>(Iin);
    const Real *l1 = static_cast<const Real *>(lamI1);
    Real *psi = static_cast<Real *>(work);
    // lanes per cell: the narrowest group (fewest lanes repeating the
    // per-cell work) whose directions-per-lane, at most 11, keep the
    // per-direction state and the prefetched next cell in registers
    const int N = G.nang;
    int sw = N <= 176 ? 16 : (N <= 352 ? 32 : 64);
    const size_t tab = (size_t)4 * N * sizeof(double);   // unit vectors and solid angles
    int cnc = (N + sw - 1) / sw;
#define RT_LAUNCH(SW, NC, RC)                                                                  \
    if (sw == SW && cnc == NC)                                                                 \
        hipLaunchKernelGGL((k_adj_couple<Real, SW, NC, RC>), dim3(nblk), dim3(kBlock), tab, s, \
                           G, in, Tin, rho, u, ka, ks, dt, l1, lamT1, psi, lamT0, gka, gks,    \
                           static_cast<const Real *>(Istar));                                  \
    else
    if (Istar) {
        RT_LAUNCH(16, 1, false) RT_LAUNCH(16, 2, false) RT_LAUNCH(16, 3, false)
        RT_LAUNCH(16, 4, false) RT_LAUNCH(16, 5, false) RT_LAUNCH(16, 6, false)
        RT_LAUNCH(16, 7, false) RT_LAUNCH(16, 8, false) RT_LAUNCH(16, 9, false)
        RT_LAUNCH(16, 10, false) RT_LAUNCH(16, 11, false)
        RT_LAUNCH(32, 6, false) RT_LAUNCH(32, 7, false) RT_LAUNCH(32, 8, false)
        RT_LAUNCH(32, 9, false) RT_LAUNCH(32, 10, false) RT_LAUNCH(32, 11, false)
        RT_LAUNCH(64, 6, false) RT_LAUNCH(64, 7, false) RT_LAUNCH(64, 8, false)
        RT_LAUNCH(64, 9, false) RT_LAUNCH(64, 10, false) RT_LAUNCH(64, 11, false)
        return RT_EINVAL;
    } else {
        // the recompute carries the transport's registers: one cell per wavefront
        sw = 64;
        cnc = (N + 63) / 64;
        RT_LAUNCH(64, 1, true) RT_LAUNCH(64, 2, true) RT_LAUNCH(64, 3, true)
        RT_LAUNCH(64, 4, true) RT_LAUNCH(64, 5, true) RT_LAUNCH(64, 6, true)
        RT_LAUNCH(64, 7, true) RT_LAUNCH(64, 8, true)
        return RT_EINVAL;
    }
#undef RT_LAUNCH
    if (hipGetLastError() != hipSuccess) return RT_EDEVICE;
    if (g->march.enabled) return launch_adj_march(g, s, Iin, psi, dt, lum_weight, lamI0);
    if (g->column.enabled) return launch_adj_column(g, s, Iin, psi, dt, lum_weight, lamI0);
#define RT_LAUNCH2(NC)                                                                         \
    case NC:                                                                                   \
        hipLaunchKernelGGL((k_adj_transport<Real, NC>), dim3(nblk), dim3(kBlock), 0, s, G, in,    \
                           static_cast<const Real *>(psi), dt, lum_weight,                      \
                           static_cast<Real *>(lamI0));                                         \
        break;
    switch (nch) {
        RT_LAUNCH2(1)
        RT_LAUNCH2(2)
        RT_LAUNCH2(3)
        RT_LAUNCH2(4)
        RT_LAUNCH2(5)
        RT_LAUNCH2(6)
        RT_LAUNCH2(7)
        RT_LAUNCH2(8)
        default:
            return RT_EINVAL;
    }
#undef RT_LAUNCH2
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

}  // namespace

int launch_adjoint(rt_grid *g, hipStream_t s, const void *Iin, const double *Tin,
                   const double *rho, const double *u, const double *ka, const double *ks,
                   double dt, double lum_weight, const void *lamI1, const double *lamT1,
                   void *lamI0, double *lamT0, void *work, double *gka, double *gks,
                   const void *Istar) {
    if (g->precision == RT_F32)
        return launch_adj_t<float>(g, s, Iin, Tin, rho, u, ka, ks, dt, lum_weight, lamI1, lamT1,
                                   lamI0, lamT0, work, gka, gks, Istar);
    return launch_adj_t<double>(g, s, Iin, Tin, rho, u, ka, ks, dt, lum_weight, lamI1, lamT1,
                                lamI0, lamT0, work, gka, gks, Istar);
}

}  // namespace rt
