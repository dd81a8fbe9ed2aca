// Fused radiation step for gfx950 (paper Sec. 2): transport (Sec. 2.3-2.4,
// 2.6) and implicit coupling (Sec. 2.5) in one pass over the intensities.
//
// Mapping: one 64-lane wavefront owns one spatial cell at a time; lane l
// handles directions l, l+64, ... (NCH chunks).  The coupling's per-cell
// angle sums are FP64 wavefront reductions, so all directions of a cell stay
// in one wave and no cross-workgroup traffic is needed.  Boundary values are
// produced from the boundary conditions inside the kernel (no ghost cells in
// memory).  Per-block partial sums (luminosity, masked energy, quartic
// failures) are reduced by a single-block finaliser in a fixed order, so
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "k_transport.h"

namespace rt {
namespace {

// Per-block partial sums of rt_step_noalloc: a file-scope device array, one
// copy on every GPU the library runs on, held until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in); it looks up each device's address once and passes that.  Every
// block writes its own slots before the finaliser reads them, so nothing has
// to be cleared between calls; calls that overlap on one GPU share the array
// and race.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kScratchDevices] = {};

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kCellsPerBlock = 16;

// LDS written by some lanes of a wavefront and read by others: order the
// accesses within the wave (no workgroup barrier; waves run different cells)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ double wave_sum(double x) { return group_sum<kWave>(x); }
__device__ __forceinline__ int wave_sum_i(int x) { return group_sum_i<kWave>(x); }

// One stage of the step: Q* = gI q I + gB q Ib - beta dt (flux terms); the
// coupling starts from gT T + gTb Tb (T alone without Tb) and runs over
// beta dt; the bookkeeping and the masked-energy ledger are weighted by wS.
// The one-stage step is {nullptr, nullptr, 1, 0, 1, 1, 0, 1}.
template <typename Real>
struct Stage {
    const Real *Ib;
    const double *Tb;
    double gI, gB, beta, gT, gTb, wS;
};

// EXT = false compiles the plain one-stage step (no stage weights, no
// optical-depth-aware flux, no velocity substitute) with the register budget
// of the general-geometry case; EXT = true carries these options.
// ANG: angular reconstruction 0 = DC, 1 = PLM, 2 = MAPR, compiled separately
// so that each option pays only for its own registers.
template <typename Real, int NCH, bool EXT, int ANG>
__device__ __forceinline__ void step_body(DevGrid G, const Real *__restrict__ Iin,
                                          Real *__restrict__ Iout, double *__restrict__ T,
                                          const double *__restrict__ rho,
                                          const double *__restrict__ uvec,
                                          const double *__restrict__ kap_a,
                                          const double *__restrict__ kap_s, double dt,
                                          double *__restrict__ dT0, double *__restrict__ partials,
                                          int *__restrict__ nr_partial, Real *__restrict__ Istar,
                                          Stage<Real> st) {
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const long long ncell = (long long)G.n0 * G.n1 * G.n2;
    const int N = G.nang;
    const Real *q = static_cast<const Real *>(G.q);
    const Real *vw = static_cast<const Real *>(G.vw);
    const Real *invV = static_cast<const Real *>(G.invV);
    const double dts = EXT ? st.beta * dt : dt;   // this stage's time step
    const Real dtR = Real(dts);
    const bool tau_on = EXT && G.tau_coeff > 0.0;
    double lum_acc = 0.0, me_acc = 0.0;
    int nr_acc = 0;
    // angular-edge records of every direction, staged once per workgroup
    __shared__ int s_adj[kMaxAngGeneral * kMaxNbr];
    // MAPR gradients, 2 N values per wave (dynamic; empty without MAPR)
    extern __shared__ __align__(16) unsigned char s_dyn[];
    if (G.has_edges) {
        for (int i = threadIdx.x; i < N * kMaxNbr; i += kBlock) s_adj[i] = edge_record(G, i);
        __syncthreads();
    }

    for (int cw = wave; cw < kCellsPerBlock; cw += kWavesPerBlock) {
        const long long cc = (long long)blockIdx.x * kCellsPerBlock + cw;
        if (cc >= ncell) break;
        const Cell x = make_cell(G, cc);
        const Real ivol = invV[x.gc];

        Real Is[NCH];
        // ---------------------------------------------------------- transport
        // axis by axis (one axis's rows live at a time), every direction of
        // the lane; then angular fluxes, primitives and the mask
        const Real *own = Iin + x.c * N;
        Real dq[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) dq[ch] = Real(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            AxisRows<Real> R;
            axis_rows(G, Iin, x, a, R);
            if (tau_on) {
                // the optical depth uses the full step in every stage
                axis_fluid(G, x, a, rho, uvec, kap_a, kap_s, dt, R);
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lane + kWave * ch;
                    if (n < N) dq[ch] += axis_div<true, Real, true>(G, R, own[n], n, lum_acc);
                }
            } else if (R.ghost) {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lane + kWave * ch;
                    if (n < N) dq[ch] += axis_div<true>(G, R, own[n], n, lum_acc);
                }
            } else {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int n = lane + kWave * ch;
                    if (n < N) dq[ch] += axis_div<false>(G, R, own[n], n, lum_acc);
                }
            }
        }
        Real *grad = reinterpret_cast<Real *>(s_dyn) + (size_t)wave * 2 * N;
        constexpr int arec = ANG;
        if constexpr (arec == 2) {
            // MAPR: every direction's gradient first, shared through LDS
            wave_sync();
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lane + kWave * ch;
                if (n >= N) continue;
                Real gx, gy;
                mapr_gradient(G, own, n, gx, gy);
                grad[2 * n] = gx;
                grad[2 * n + 1] = gy;
            }
            wave_sync();
        }
        {
            const Real *qrow = q + (size_t)x.gc * N;
            const uint8_t *mrow = G.mask + (size_t)x.gc * N;
            const Real *vwrow = vw + (size_t)x.gc * G.nedge * 2;
            const double volD = G.volD[x.gc];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lane + kWave * ch;
                Is[ch] = Real(0);
                if (n >= N) continue;
                const Real Ic = own[n];
                const Real div = !G.has_edges ? Real(0)
                                 : (arec == 2 ? angular_div_mapr(G, s_adj, own, vwrow, grad, n)
                                    : arec == 1 ? angular_div_plm(G, s_adj, own, vwrow, n)
                                                       : angular_div_rec(s_adj, own, vwrow, n));
                const Real qn = qrow[n];
                Real Qs = qn * Ic;
                if (EXT && st.Ib) Qs = Real(st.gI) * Qs + Real(st.gB) * (qn * st.Ib[x.c * N + n]);
                Qs = Qs - dtR * ivol * dq[ch] - quot(dtR * div, Real(G.domega[n]));
                if (mrow[n]) {
                    me_acc -= (EXT ? st.wS : 1.0) * volD * G.domega[n] * (double)Qs;
                    continue;
                }
                Is[ch] = quot(Qs, qn);
            }
        }
        if (Istar) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lane + kWave * ch;
                if (n < N) Istar[x.c * N + n] = Is[ch];
            }
        }

        // ---------------------------------------------------------- coupling
        // per direction nb = n^0bar, dn = n^0 + nb tau, rr = 1/(nb^2 dn); the
        // quotients n^0/dn, 1/(nb dn), 1/(dn nb^3) are products with rr
        double u1 = uvec[3 * x.c], u2 = uvec[3 * x.c + 1], u3 = uvec[3 * x.c + 2];
        double u0 = sqrt(fma(u1, u1, fma(u2, u2, fma(u3, u3, 1.0))));
        const double rh = rho[x.c];
        const double aa = kap_a[x.c] * rh, as = kap_s[x.c] * rh;
        const double tau = (aa + as) * dts;
        const double n0 = G.n0u[x.gc];
        const uint8_t *mrow = G.mask + (size_t)x.gc * N;
        const double Tm = (EXT && st.Tb) ? st.gT * T[x.c] + st.gTb * st.Tb[x.c] : T[x.c];
        if (EXT && G.rad_velocity) {
            // radiation-dominated velocity substitute (Sec. 2.5): with the gas
            // velocity, E = sum I n0bar^2 dOm, R^00, R^0a and sum n^a n0bar I dOm
            // (= -u_b R^ab); cells with E > rho + u_gas couple at the blend
            double sv[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int n = lane + kWave * ch;
                if (n >= N || mrow[n]) continue;
                const double nx = G.nhat[3 * n], ny = G.nhat[3 * n + 1], nz = G.nhat[3 * n + 2];
                const double nb = u0 - fma(u1, nx, fma(u2, ny, u3 * nz));
                const double Iw = (double)Is[ch] * G.domega[n];
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
            velocity_substitute(sv, rh, Tm, aa, as, n0, dts, G.cv, G.kb, G.a_rad, u0, u1, u2, u3);
        }
        double nbv[NCH], rrv[NCH];
        double sf[3] = {0.0, 0.0, 0.0};   // Em, A1, A2
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = lane + kWave * ch;
            const int m = n < N ? n : 0;
            const double nb = u0 - fma(u1, G.nhat[3 * m], fma(u2, G.nhat[3 * m + 1], u3 * G.nhat[3 * m + 2]));
            const double nb2 = nb * nb;
            const double rr = rcp64(nb2 * fma(nb, tau, n0));
            nbv[ch] = nb;
            rrv[ch] = rr;
            if (n >= N || mrow[n]) continue;
            const double dom = G.domega[n];
            const double Iw = (double)Is[ch] * (nb2 * dom);
            sf[0] += Iw;
            sf[1] = fma(n0 * nb2 * rr, Iw, sf[1]);
            sf[2] = fma(dom, nb * rr, sf[2]);
        }
        wave_sum_quads(sf);
        const double Em = sf[0], A1 = sf[1], A2 = sf[2] * (dts / kFourPi);
        const double B4 = A2 * aa * G.a_rad;
        const double B1 = rh * G.cv * (1.0 - A2 * as);
        const double B0 = A1 - B1 * Tm - (1.0 - A2 * as) * Em;
        int bad = 0;
        const double Tp = quartic_root_fast(B4, B1, B0, bad, Tm);
        const double Ep = Em - rh * G.cv * (Tp - Tm);
        const double Tp2 = Tp * Tp;
        const double S = aa * G.a_rad * Tp2 * Tp2 + as * Ep;
        const double cS = S * (dts / kFourPi);
        double sm[4] = {0.0, 0.0, 0.0, 0.0};
        const bool beam_cell = G.beam != nullptr && G.beam[x.c];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int n = lane + kWave * ch;
            if (n >= N) continue;
            Real out = Real(0);
            if (!mrow[n]) {
                const double nb = nbv[ch], rr = rrv[ch];
                const double nbrr = nb * rr;                       // 1/(nb dn)
                const double dn = fma(nb, tau, n0);
                const double I = (double)Is[ch];
                // I+ = (n^0/dn) I* + dt S / (4 pi dn nb^3)
                const double Ip = fma(n0 * nb * nbrr, I, cS * (nbrr * rr * dn));
                const double dI = (Ip - I) * G.domega[n];
                sm[0] += dI;
                sm[1] = fma(dI, G.nhat[3 * n], sm[1]);
                sm[2] = fma(dI, G.nhat[3 * n + 1], sm[2]);
                sm[3] = fma(dI, G.nhat[3 * n + 2], sm[3]);
                out = Real(Ip);
            }
            if (beam_cell && n == G.beam_angle) out = Real(G.beam_I);
            Iout[x.c * N + n] = out;
        }
        if (lane == 0) {
            T[x.c] = Tp;
            nr_acc += bad;
        }
        if (dT0) {
            wave_sum_quads(sm);
            if (lane == 0) {
                const double *E0 = G.E0 + 16 * x.gc;
#pragma unroll
                for (int al = 0; al < 4; ++al)
                    dT0[4 * x.c + al] -= (EXT ? st.wS : 1.0) * n0 * (E0[4 * al] * sm[0] + E0[4 * al + 1] * sm[1] +
                                                       E0[4 * al + 2] * sm[2] + E0[4 * al + 3] * sm[3]);
            }
        }
    }
    // -------------------------------------------------------- block partials
    __shared__ double sh_l[kWavesPerBlock], sh_m[kWavesPerBlock];
    __shared__ int sh_n[kWavesPerBlock];
    lum_acc = wave_sum(lum_acc);
    me_acc = wave_sum(me_acc);
    nr_acc = wave_sum_i(nr_acc);
    if (lane == 0) {
        sh_l[wave] = lum_acc;
        sh_m[wave] = me_acc;
        sh_n[wave] = nr_acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double l = 0.0, m = 0.0;
        int r = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            l += sh_l[w];
            m += sh_m[w];
            r += sh_n[w];
        }
        partials[2 * blockIdx.x] = l;
        partials[2 * blockIdx.x + 1] = m;
        nr_partial[blockIdx.x] = r;
    }
}

#define RT_STEP_ARGS                                                                           \
    DevGrid G, const Real *__restrict__ Iin, Real *__restrict__ Iout, double *__restrict__ T,  \
        const double *__restrict__ rho, const double *__restrict__ uvec,                       \
        const double *__restrict__ kap_a, const double *__restrict__ kap_s, double dt,         \
        double *__restrict__ dT0, double *__restrict__ partials, int *__restrict__ nr_partial, \
        Real *__restrict__ Istar, Stage<Real> st
#define RT_STEP_PASS G, Iin, Iout, T, rho, uvec, kap_a, kap_s, dt, dT0, partials, nr_partial, Istar, st

template <typename Real, int NCH, bool EXT, int ANG = 0>
__global__ __launch_bounds__(kBlock) void k_step(RT_STEP_ARGS) {
    step_body<Real, NCH, EXT, ANG>(RT_STEP_PASS);
}

// The plain step of up to six direction chunks under a tighter register
// budget (five waves per SIMD up to three chunks, four up to six): more waves
// hide more of the latency of its neighbour and geometry gathers (about 6%
// faster on the 128 x 64 x 128 x 162 Kerr-Schild grid, 12% on 256 x 128 x
// 256 x 362).
template <typename Real, int NCH, int ANG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NCH <= 3 ? 5 : 4))) void k_step_lean(
    RT_STEP_ARGS) {
    step_body<Real, NCH, false, ANG>(RT_STEP_PASS);
}
#undef RT_STEP_ARGS
#undef RT_STEP_PASS

// Single-block, fixed-order reduction of the per-block partials.
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ partials,
                                                     const int *__restrict__ nr_partial,
                                                     int nblocks, double dt, double *lum,
                                                     double *ledger, long long *noroot) {
    __shared__ double sl[kBlock], sm[kBlock];
    __shared__ long long sn[kBlock];
    double l = 0.0, m = 0.0;
    long long r = 0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
        l += partials[2 * b];
        m += partials[2 * b + 1];
        r += nr_partial[b];
    }
    sl[threadIdx.x] = l;
    sm[threadIdx.x] = m;
    sn[threadIdx.x] = r;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sl[threadIdx.x] += sl[threadIdx.x + s];
            sm[threadIdx.x] += sm[threadIdx.x + s];
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (lum) *lum += dt * sl[0];
        *ledger += sm[0];
        *noroot += sn[0];
    }
}

// Per-cell moments: one wave per cell, FP64 sums over directions.
template <typename Real>
__global__ __launch_bounds__(kBlock) void k_moments(DevGrid G, const Real *__restrict__ I,
                                                    const double *__restrict__ uvec,
                                                    double *__restrict__ R,
                                                    double *__restrict__ R0,
                                                    double *__restrict__ E) {
    const int lane = threadIdx.x % kWave;
    const long long ncell = (long long)G.n0 * G.n1 * G.n2;
    const long long c = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (c >= ncell) return;
    const int N = G.nang;
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int n = lane; n < N; n += kWave) {
        const double w = (double)I[c * N + n] * G.domega[n];
        const double x = G.nhat[3 * n], y = G.nhat[3 * n + 1], z = G.nhat[3 * n + 2];
        s[0] += w;
        s[1] += w * x;
        s[2] += w * y;
        s[3] += w * z;
        s[4] += w * x * x;
        s[5] += w * x * y;
        s[6] += w * x * z;
        s[7] += w * y * y;
        s[8] += w * y * z;
        s[9] += w * z * z;
    }
    group_sum_v<kWave, 10>(s);
    if (lane != 0) return;
    if (R)
        for (int m = 0; m < 10; ++m) R[10 * c + m] = s[m];
    const int i = (int)(c % G.n0), j = (int)((c / G.n0) % G.n1), k = (int)(c / ((long long)G.n0 * G.n1));
    const int gc = ((G.g2 > 1 ? k : 0) * G.g1 + (G.g1 > 1 ? j : 0)) * G.g0 + (G.g0 > 1 ? i : 0);
    if (R0) {
        const double *E0 = G.E0 + 16 * gc;
        const double n0 = G.n0u[gc];
        for (int al = 0; al < 4; ++al)
            R0[4 * c + al] = n0 * (E0[4 * al] * s[0] + E0[4 * al + 1] * s[1] + E0[4 * al + 2] * s[2] +
                                   E0[4 * al + 3] * s[3]);
    }
    if (E) {
        const double u1 = uvec[3 * c], u2 = uvec[3 * c + 1], u3 = uvec[3 * c + 2];
        const double u0 = sqrt(1.0 + u1 * u1 + u2 * u2 + u3 * u3);
        // sum I (u0 - u.n)^2 dOmega from the ten moments
        E[c] = u0 * u0 * s[0] - 2.0 * u0 * (u1 * s[1] + u2 * s[2] + u3 * s[3]) +
               u1 * u1 * s[4] + 2.0 * u1 * u2 * s[5] + 2.0 * u1 * u3 * s[6] + u2 * u2 * s[7] +
               2.0 * u2 * u3 * s[8] + u3 * u3 * s[9];
    }
}

template <typename Real>
int launch_step_t(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                  const double *rho, const double *u, const double *ka, const double *ks,
                  double dt, double *dT0, double *lum, void *Istar, const Stage<Real> &st,
                  double lum_dt, const Partials &P) {
    const DevGrid &G = g->dg;
    const int nblk = step_blocks(g);
    const int nch = (G.nang + kWave - 1) / kWave;
    const Real *in = static_cast<const Real *>(Iin);
    Real *out = static_cast<Real *>(Iout);
    const bool ext = g->integrator == 2 || G.tau_coeff > 0.0 || G.rad_velocity;
    const size_t lds = G.ang_recon == 2 ? (size_t)kWavesPerBlock * 2 * G.nang * sizeof(Real) : 0;
#define RT_LAUNCH_A(NC, E, A)                                                                  \
    hipLaunchKernelGGL((k_step<Real, NC, E, A>), dim3(nblk), dim3(kBlock), lds, s, G, in, out,    \
                       T, rho, u, ka, ks, dt, dT0, P.sums, P.noroot,                           \
                       static_cast<Real *>(Istar), st)
#define RT_LAUNCH_E(NC, E)                                                                     \
    if (G.ang_recon == 2)                                                                      \
        RT_LAUNCH_A(NC, E, 2);                                                                 \
    else if (G.ang_recon == 1)                                                                 \
        RT_LAUNCH_A(NC, E, 1);                                                                 \
    else                                                                                       \
        RT_LAUNCH_A(NC, E, 0);
#define RT_LAUNCH(NC)                                                                          \
    case NC:                                                                                   \
        if (ext) {                                                                             \
            RT_LAUNCH_E(NC, true)                                                              \
        } else if (NC <= 6 && G.ang_recon != 2) {                                              \
            if (G.ang_recon == 1)                                                              \
                hipLaunchKernelGGL((k_step_lean<Real, NC, 1>), dim3(nblk), dim3(kBlock), lds, s, \
                                   G, in, out, T, rho, u, ka, ks, dt, dT0, P.sums,             \
                                   P.noroot, static_cast<Real *>(Istar), st);                  \
            else                                                                               \
                hipLaunchKernelGGL((k_step_lean<Real, NC, 0>), dim3(nblk), dim3(kBlock), lds, s, \
                                   G, in, out, T, rho, u, ka, ks, dt, dT0, P.sums,             \
                                   P.noroot, static_cast<Real *>(Istar), st);                  \
        } else {                                                                               \
            RT_LAUNCH_E(NC, false)                                                             \
        }                                                                                      \
        break;
    switch (nch) {
        RT_LAUNCH(1)
        RT_LAUNCH(2)
        RT_LAUNCH(3)
        RT_LAUNCH(4)
        RT_LAUNCH(5)
        RT_LAUNCH(6)
        RT_LAUNCH(7)
        RT_LAUNCH(8)
        default:
            return RT_EINVAL;
    }
#undef RT_LAUNCH
#undef RT_LAUNCH_A
#undef RT_LAUNCH_E
    if (hipGetLastError() != hipSuccess) return RT_EDEVICE;
    return launch_finalize(g, s, nblk, lum_dt, lum, P);
}

// The two-stage (Heun) step: stage 1 into the grid's stage buffers, stage 2
// from them (and from I_in, T) into I_out, T.
template <typename Real>
int launch_rk2_t(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                 const double *rho, const double *u, const double *ka, const double *ks,
                 double dt, double *dT0, double *lum, const Partials &P) {
    const size_t ncell = (size_t)g->dg.n0 * g->dg.n1 * g->dg.n2;
    if (hipMemcpyAsync(g->stage_T, T, ncell * sizeof(double), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return RT_EDEVICE;
    const Stage<Real> s1{nullptr, nullptr, 1.0, 0.0, 1.0, 1.0, 0.0, 0.5};
    int rc = launch_step_t<Real>(g, s, Iin, g->stage_I, g->stage_T, rho, u, ka, ks, dt, dT0, lum,
                                 nullptr, s1, 0.5 * dt, P);
    if (rc != RT_OK) return rc;
    const Stage<Real> s2{static_cast<const Real *>(Iin), g->stage_T, 0.5, 0.5, 0.5, 0.5, 0.5, 1.0};
    return launch_step_t<Real>(g, s, g->stage_I, Iout, T, rho, u, ka, ks, dt, dT0, lum, nullptr,
                               s2, 0.5 * dt, P);
}

}  // namespace

int step_blocks(const rt_grid *g) {
    const long long ncell = (long long)g->dg.n0 * g->dg.n1 * g->dg.n2;
    return (int)((ncell + kCellsPerBlock - 1) / kCellsPerBlock);
}

int step_partial_blocks(const rt_grid *g) {
    if (g->march.enabled) return g->march.grid;
    if (g->column.enabled) return g->column.grid;
    return step_blocks(g);
}

int scratch_address(void **ptr, size_t *bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return RT_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RT_EDEVICE;
        g_scratch_addr[dev] = p;
    }
    *ptr = g_scratch_addr[dev];
    *bytes = kScratchBytes;
    return RT_OK;
}

// Dynamic-LDS limit of a kernel on the current device: raised once per
// (device, kernel) to `bytes` (or more), under a lock, before its first
// launch on that device.
namespace {
std::mutex g_lds_mu;
std::map<std::pair<int, const void *>, int> g_lds_limit;
}  // namespace

int ensure_dynamic_lds(const void *kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return RT_OK;   // within the default limit
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RT_EDEVICE;
    std::lock_guard<std::mutex> lock(g_lds_mu);
    int &cur = g_lds_limit[{dev, kernel}];
    if (cur >= (int)bytes) return RT_OK;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
        hipSuccess)
        return RT_EDEVICE;
    cur = (int)bytes;
    return RT_OK;
}

int launch_finalize(rt_grid *g, hipStream_t s, int nblocks, double dt, double *lum,
                    const Partials &P) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, P.sums, P.noroot, nblocks, dt,
                       lum, g->ledger, g->noroot);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

int launch_step(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                const double *rho, const double *u, const double *ka, const double *ks,
                double dt, double *dT0, double *lum, void *Istar, const Partials &P) {
    if (g->march.enabled && g->integrator == 2)
        return launch_march_rk2(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
    if (g->march.enabled) {
        int rc = launch_march(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
        if (rc != RT_OK) return rc;
        return launch_finalize(g, s, g->march.grid, dt, lum, P);
    }
    if (g->column.enabled && g->integrator == 2)
        return launch_column_rk2(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
    if (g->column.enabled) {
        int rc = launch_column(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, Istar, P);
        if (rc != RT_OK) return rc;
        return launch_finalize(g, s, g->column.grid, dt, lum, P);
    }
    if (g->integrator == 2) {
        if (g->precision == RT_F32)
            return launch_rk2_t<float>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
        return launch_rk2_t<double>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, P);
    }
    if (g->precision == RT_F32)
        return launch_step_t<float>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, Istar,
                                    Stage<float>{nullptr, nullptr, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0}, dt,
                                    P);
    return launch_step_t<double>(g, s, Iin, Iout, T, rho, u, ka, ks, dt, dT0, lum, Istar,
                                 Stage<double>{nullptr, nullptr, 1.0, 0.0, 1.0, 1.0, 0.0, 1.0}, dt,
                                 P);
}

int launch_moments(rt_grid *g, hipStream_t s, const void *I, const double *u, double *R,
                   double *R0, double *E) {
    const long long ncell = (long long)g->dg.n0 * g->dg.n1 * g->dg.n2;
    const int nblk = (int)((ncell + kWavesPerBlock - 1) / kWavesPerBlock);
    if (g->precision == RT_F32)
        hipLaunchKernelGGL(k_moments<float>, dim3(nblk), dim3(kBlock), 0, s, g->dg,
                           static_cast<const float *>(I), u, R, R0, E);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(nblk), dim3(kBlock), 0, s, g->dg,
                           static_cast<const double *>(I), u, R, R0, E);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

}  // namespace rt
