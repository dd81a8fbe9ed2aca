// C ABI of the radiation step: validation, table upload, scratch, dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <limits>
#include <new>
#include <sstream>
#include <string>

#include "k_tile.h"
#include "rt_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

struct Uploader {
    rt_grid *g;
    int code = RT_OK;
    std::string msg;
    template <typename T>
    T *put(const T *src, size_t count) {
        if (code != RT_OK) return nullptr;
        void *p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            code = RT_ENOMEM;
            msg = "hipMalloc failed for a geometry table";
            return nullptr;
        }
        g->allocs.push_back(p);
        if (count && hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
            code = RT_EDEVICE;
            msg = "hipMemcpy of a geometry table failed";
            return nullptr;
        }
        return static_cast<T *>(p);
    }
    template <typename T>
    T *zeros(size_t count) {
        if (code != RT_OK) return nullptr;
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
            code = RT_ENOMEM;
            msg = "hipMalloc failed for scratch";
            return nullptr;
        }
        g->allocs.push_back(p);
        if (hipMemset(p, 0, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
            code = RT_EDEVICE;
            msg = "hipMemset of scratch failed";
        }
        return static_cast<T *>(p);
    }
    // geometry coefficients in the intensity precision
    const void *real(const std::vector<double> &v, int precision) {
        if (precision == RT_F64) return put(v.data(), v.size());
        std::vector<float> f(v.begin(), v.end());
        return put(f.data(), f.size());
    }
};

void release(rt_grid *g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    for (void *p : g->allocs) (void)hipFree(p);
    g->allocs.clear();
    (void)hipSetDevice(cur);
}

}  // namespace

extern "C" {

const char *rt_last_error(void) { return g_err.c_str(); }

int rt_init_grid(const rt_grid_desc *d, int device, rt_grid **out) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    *out = nullptr;
    std::string derr;
    int rc = rt::check_desc(d, derr);
    if (rc != RT_OK) return fail(rc, derr);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(RT_EDEVICE, "no such HIP device");
    rt_grid *g = nullptr;
    try {
        g = new rt_grid();
        g->device = device;
        g->precision = d->precision;
        g->ang = d->n_zeta > 0 ? rt::build_latlong(d->n_zeta, d->n_psi) : rt::build_geodesic(d->nlev);
        rt::HostTables t;
        std::string err;
        rc = rt::build_tables(*d, g->ang, t, err);
        if (rc != RT_OK) {
            delete g;
            return fail(rc, err);
        }
        const int N = g->ang.nang, E = g->ang.nedge;
        const int G = t.G;
        // host copies for rt_max_dt
        for (int a = 0; a < 3; ++a) {
            g->dx[a].resize(d->n[a]);
            for (int i = 0; i < d->n[a]; ++i) g->dx[a][i] = d->x_faces[a][i + 1] - d->x_faces[a][i];
        }
        g->host_n0u = t.n0u;
        g->host_vw = t.vw;
        g->host_na.assign((size_t)G * N * 3, 0.0);
        for (int c = 0; c < G; ++c) {
            const double *e = d->tet_c + 16 * c;
            for (int n = 0; n < N; ++n) {
                const double *nh = &g->ang.nhat[3 * n];
                for (int a = 0; a < 3; ++a)
                    g->host_na[((size_t)c * N + n) * 3 + a] =
                        e[4 * (a + 1)] + e[4 * (a + 1) + 1] * nh[0] + e[4 * (a + 1) + 2] * nh[1] +
                        e[4 * (a + 1) + 3] * nh[2];
            }
        }
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (hipSetDevice(device) != hipSuccess) {
            delete g;
            return fail(RT_EDEVICE, "hipSetDevice failed");
        }
        Uploader up{g};
        rt::DevGrid &v = g->dg;
        v.n0 = d->n[0];
        v.n1 = d->n[1];
        v.n2 = d->n[2];
        v.nang = N;
        v.nedge = E;
        v.g0 = d->geo_extent[0];
        v.g1 = d->geo_extent[1];
        v.g2 = d->geo_extent[2];
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b)
                v.fe[a][b] = (b == a) ? (d->geo_extent[b] > 1 ? d->n[b] + 1 : 1) : d->geo_extent[b];
            v.bc[a][0] = d->bc[a][0];
            v.bc[a][1] = d->bc[a][1];
        }
        v.recon = d->recon;
        v.lum_axis = d->lum_axis;
        v.lum_side = d->lum_side;
        v.a_rad = d->a_rad;
        v.cv = d->kb_mu_mp / (d->gamma_gas - 1.0);
        v.tau_coeff = d->tau_coeff;
        v.kb = d->kb_mu_mp;
        v.gamma = d->gamma_gas;
        v.rad_velocity = d->rad_velocity ? 1 : 0;
        g->integrator = d->integrator == 2 ? 2 : 1;
        v.nhat = up.put(g->ang.nhat.data(), g->ang.nhat.size());
        v.domega = up.put(g->ang.domega.data(), g->ang.domega.size());
        v.adj_e = up.put(g->ang.adj_e.data(), g->ang.adj_e.size());
        v.adj_s = up.put(g->ang.adj_s.data(), g->ang.adj_s.size());
        v.edge_lo = up.put(g->ang.lo.data(), g->ang.lo.size());
        v.edge_hi = up.put(g->ang.hi.data(), g->ang.hi.size());
        v.ang_recon = d->ang_recon;
        v.edge_ll = g->ang.ll.empty() ? nullptr : up.put(g->ang.ll.data(), g->ang.ll.size());
        v.edge_rr = g->ang.rr.empty() ? nullptr : up.put(g->ang.rr.data(), g->ang.rr.size());
        v.mapr_nb = nullptr;
        v.mapr_cnt = nullptr;
        v.mapr_inv = nullptr;
        v.mapr_d = nullptr;
        if (d->ang_recon == 2) {
            std::vector<int> nb;
            std::vector<double> inv, dd;
            std::vector<int8_t> cnt;
            rt::build_mapr(g->ang, nb, inv, cnt, dd);
            v.mapr_nb = up.put(nb.data(), nb.size());
            v.mapr_cnt = up.put(cnt.data(), cnt.size());
            v.mapr_inv = up.real(inv, d->precision);
            v.mapr_d = up.real(dd, d->precision);
        }
        v.q = up.real(t.q, d->precision);
        for (int a = 0; a < 3; ++a) {
            v.C[a] = up.real(t.C[a], d->precision);
            v.sgn[a] = up.put(t.sgn[a].data(), t.sgn[a].size());
        }
        v.vw = up.real(t.vw, d->precision);
        std::vector<double> invV(G);
        for (int c = 0; c < G; ++c) invV[c] = 1.0 / t.vol[c];
        v.invV = up.real(invV, d->precision);
        v.mask = up.put(t.mask.data(), t.mask.size());
        v.n0u = up.put(t.n0u.data(), t.n0u.size());
        v.E0 = up.put(t.E0.data(), t.E0.size());
        v.gas_map = up.put(t.gas_map.data(), t.gas_map.size());
        v.volD = up.put(t.vol.data(), t.vol.size());
        v.has_edges = t.has_edges ? 1 : 0;
        const size_t ncell = (size_t)d->n[0] * d->n[1] * d->n[2];
        if (d->beam_mask) {
            v.beam = up.put(d->beam_mask, ncell);
            v.beam_angle = d->beam_angle;
            v.beam_I = d->beam_I;
        } else {
            v.beam = nullptr;
            v.beam_angle = -1;
            v.beam_I = 0.0;
        }
        // fast path for spatially uniform geometry
        {
            rt::MarchInfo &M = g->march;
            M.enabled = 0;
            M.any_mask = 0;
            int sw = 0, nc = 0;
            const bool allow = d->kernel != 1;
            const bool cfg = rt::march_config(d->precision, N, sw, nc);
            const size_t lds = cfg ? rt::march_lds_bytes(d->precision, N, sw * nc) : 0;
            if (allow && cfg && G == 1 && !t.has_edges &&
                (g->integrator == 1 || rt::march_rk2_config(sw, nc)) &&
                !(d->tau_coeff > 0.0) && !d->rad_velocity && d->n[0] % rt::kTX == 0 &&
                d->n[1] % rt::kTY == 0 &&
                lds <= 150 * 1024) {
                std::vector<double> q(N), iq(N), cx(N), cy(N), cz(N);
                std::vector<uint8_t> bits(N, 0);
                for (int n = 0; n < N; ++n) {
                    q[n] = t.q[n];
                    iq[n] = 1.0 / t.q[n];
                    // flux coefficients C/dV with the sign of the motion folded in
                    cx[n] = (t.sgn[0][n] < 0 ? -1.0 : 1.0) * t.C[0][n] * invV[0];
                    cy[n] = (t.sgn[1][n] < 0 ? -1.0 : 1.0) * t.C[1][n] * invV[0];
                    cz[n] = (t.sgn[2][n] < 0 ? -1.0 : 1.0) * t.C[2][n] * invV[0];
                    uint8_t b = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (t.sgn[a][n] > 0) b |= (uint8_t)(1u << (2 * a));
                        if (t.sgn[a][n] < 0) b |= (uint8_t)(2u << (2 * a));
                    }
                    if (t.mask[n]) b |= 64;
                    bits[n] = b;
                    if (t.mask[n]) M.any_mask = 1;
                }
                M.q = up.real(q, d->precision);
                M.iq = up.real(iq, d->precision);
                M.cx = up.real(cx, d->precision);
                M.cy = up.real(cy, d->precision);
                M.cz = up.real(cz, d->precision);
                M.bits = up.put(bits.data(), bits.size());
                M.vol = t.vol[0];
                M.sw = sw;
                M.nc = nc;
                M.lds = lds;
                M.pstride = rt::march_pstride(d->precision, sw * nc);
                M.ntx = d->n[0] / rt::kTX;
                const long long ntiles = (long long)(d->n[0] / rt::kTX) * (d->n[1] / rt::kTY);
                const long long target = 2048;
                long long seglen = d->seglen > 0
                                       ? d->seglen
                                       : std::max<long long>(4, (d->n[2] * ntiles + target - 1) / target);
                seglen = std::min<long long>(seglen, d->n[2]);
                M.seglen = (int)seglen;
                M.nseg = (int)((d->n[2] + seglen - 1) / seglen);
                const long long nwork = ntiles * M.nseg;
                if (nwork < (1LL << 30)) {
                    M.nwork = (int)nwork;
                    M.grid = (int)((nwork + 7) / 8 * 8);
                    M.enabled = 1;
                }
            }
        }
        // column march for geometry independent of axis 2 (one-stage step
        // with DC, PLM or MAPR angular fluxes, or DC with the velocity
        // substitute; DC with the two-stage step and/or the optical-depth-
        // aware flux)
        g->column.enabled = 0;
        if (!g->march.enabled && d->kernel != 1 && d->geo_extent[2] == 1 &&
            (g->integrator == 1 || (d->ang_recon == 0 && !d->rad_velocity)) &&
            (!(d->tau_coeff > 0.0) || (d->ang_recon == 0 && !d->rad_velocity)) &&
            (!d->rad_velocity || d->ang_recon == 0) &&
            (N + rt::kWave - 1) / rt::kWave <= rt::kMaxChunks)
            g->column.enabled = rt::column_config(g, d->seglen) ? 1 : 0;
        // this device's static scratch for rt_step_noalloc (looked up once per
        // device, with the device current); a failed lookup leaves it unset and
        // only that entry point reports it
        {
            void *sp = nullptr;
            size_t sb = 0;
            if (rt::scratch_address(&sp, &sb) == RT_OK) {
                g->scratch = sp;
                g->scratch_bytes = sb;
            }
        }
        g->max_blocks = std::max({rt::step_blocks(g), g->march.enabled ? g->march.grid : 0,
                                  g->column.enabled ? g->column.grid : 0});
        g->partials = up.zeros<double>((size_t)g->max_blocks * 2);
        g->noroot_partial = up.zeros<int>((size_t)g->max_blocks);
        g->ledger = up.zeros<double>(1);
        g->noroot = up.zeros<long long>(1);
        if (g->integrator == 2) {
            // stage-1 state of the two-stage integrator
            g->stage_I = up.zeros<unsigned char>(ncell * (size_t)N * (d->precision == RT_F32 ? 4 : 8));
            g->stage_T = up.zeros<double>(ncell);
        }
        (void)hipSetDevice(cur);
        if (up.code != RT_OK) {
            release(g);
            delete g;
            return fail(up.code, up.msg);
        }
        *out = g;
        g_err.clear();
        return RT_OK;
    } catch (const std::bad_alloc &) {
        if (g) {
            release(g);
            delete g;
        }
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        if (g) {
            release(g);
            delete g;
        }
        return fail(RT_EINVAL, ex.what());
    }
}

int rt_geodesic_angles(int32_t nlev, double *nhat, double *domega) {
    if (nlev < 1 || nlev > 7) return fail(RT_EINVAL, "nlev must be in 1..7");
    try {
        rt::Geodesic a = rt::build_geodesic(nlev);
        if (nhat) std::memcpy(nhat, a.nhat.data(), a.nhat.size() * sizeof(double));
        if (domega) std::memcpy(domega, a.domega.data(), a.domega.size() * sizeof(double));
    } catch (const std::exception &ex) {
        return fail(RT_EINVAL, ex.what());
    }
    return RT_OK;
}

int rt_latlong_angles(int32_t n_zeta, int32_t n_psi, double *nhat, double *domega) {
    if (n_zeta < 2 || n_psi < 2 || (n_psi & 1) || n_zeta * n_psi > 512)
        return fail(RT_EINVAL, "latitude-longitude grid needs n_zeta >= 2, an even n_psi >= 2 and "
                               "n_zeta n_psi <= 512");
    try {
        rt::Geodesic a = rt::build_latlong(n_zeta, n_psi);
        if (nhat) std::memcpy(nhat, a.nhat.data(), a.nhat.size() * sizeof(double));
        if (domega) std::memcpy(domega, a.domega.data(), a.domega.size() * sizeof(double));
    } catch (const std::exception &ex) {
        return fail(RT_EINVAL, ex.what());
    }
    return RT_OK;
}

int rt_grid_info(const rt_grid *g, int32_t *nang, int32_t *nedge, int32_t *fast_path) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (nang) *nang = g->ang.nang;
    if (nedge) *nedge = g->ang.nedge;
    if (fast_path) *fast_path = g->march.enabled ? 1 : (g->column.enabled ? 2 : 0);
    return RT_OK;
}

int rt_angles(const rt_grid *g, double *nhat, double *domega) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (nhat) std::memcpy(nhat, g->ang.nhat.data(), g->ang.nhat.size() * sizeof(double));
    if (domega) std::memcpy(domega, g->ang.domega.data(), g->ang.domega.size() * sizeof(double));
    return RT_OK;
}

int rt_max_dt(const rt_grid *g, double cfl, double *dt) {
    if (!g || !dt) return fail(RT_EINVAL, "NULL argument");
    if (!(cfl > 0.0)) return fail(RT_EINVAL, "cfl must be positive");
    const rt::DevGrid &v = g->dg;
    const int N = v.nang, E = v.nedge;
    double best = std::numeric_limits<double>::infinity();
    for (int gk = 0; gk < v.g2; ++gk)
        for (int gj = 0; gj < v.g1; ++gj)
            for (int gi = 0; gi < v.g0; ++gi) {
                const int c = (gk * v.g1 + gj) * v.g0 + gi;
                const double n0 = g->host_n0u[c];
                const double dxs[3] = {g->dx[0][gi], g->dx[1][gj], g->dx[2][gk]};
                std::vector<double> out(N, 0.0);
                for (int e = 0; e < E; ++e) {
                    double vv = g->host_vw[((size_t)c * E + e) * 2];
                    if (vv > 0) out[g->ang.lo[e]] += vv;
                    if (vv < 0) out[g->ang.hi[e]] += -vv;
                }
                for (int n = 0; n < N; ++n) {
                    for (int a = 0; a < 3; ++a) {
                        double na = std::fabs(g->host_na[((size_t)c * N + n) * 3 + a]);
                        if (na > 0) best = std::fmin(best, dxs[a] * n0 / na);
                    }
                    if (out[n] > 0) best = std::fmin(best, g->ang.domega[n] * n0 / out[n]);
                }
            }
    *dt = cfl * best;
    return RT_OK;
}

int rt_step(rt_grid *g, void *stream, const void *I_in, void *I_out, double *T,
            const double *rho, const double *u_tet, const double *kappa_a,
            const double *kappa_s, double dt, double *dT0, double *lum, void *I_star) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (!I_in || !I_out || !T || !rho || !u_tet || !kappa_a || !kappa_s)
        return fail(RT_EINVAL, "NULL state pointer");
    if (I_in == I_out) return fail(RT_EINVAL, "I_out must not alias I_in");
    if (I_star && (I_star == I_in || I_star == I_out))
        return fail(RT_EINVAL, "I_star must not alias I_in or I_out");
    if (I_star && (g->integrator == 2 || g->dg.tau_coeff > 0.0))
        return fail(RT_EINVAL, "I_star needs the one-stage step without the optical-depth-aware flux");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RT_EINVAL, "dt must be positive and finite");
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    int rc = rt::launch_step(g, (hipStream_t)stream, I_in, I_out, T, rho, u_tet, kappa_a, kappa_s,
                             dt, dT0, lum, I_star, rt::Partials{g->partials, g->noroot_partial});
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc != RT_OK) return fail(rc, "kernel launch failed");
    return RT_OK;
}

int rt_step_noalloc(rt_grid *g, void *stream, const void *I_in, void *I_out, double *T,
                    const double *rho, const double *u_tet, const double *kappa_a,
                    const double *kappa_s, double dt, double *dT0, double *lum, void *I_star) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (!I_in || !I_out || !T || !rho || !u_tet || !kappa_a || !kappa_s)
        return fail(RT_EINVAL, "NULL state pointer");
    if (I_in == I_out) return fail(RT_EINVAL, "I_out must not alias I_in");
    if (I_star && (I_star == I_in || I_star == I_out))
        return fail(RT_EINVAL, "I_star must not alias I_in or I_out");
    if (I_star && (g->integrator == 2 || g->dg.tau_coeff > 0.0))
        return fail(RT_EINVAL, "I_star needs the one-stage step without the optical-depth-aware flux");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RT_EINVAL, "dt must be positive and finite");
    if (!g->scratch) return fail(RT_EDEVICE, "the device's static scratch could not be located");
    // layout: [blocks][2] doubles, then [blocks] ints from the next 256-byte boundary
    const size_t nb = (size_t)rt::step_partial_blocks(g);
    const size_t off = (nb * 2 * sizeof(double) + 255) / 256 * 256;
    const size_t need = off + nb * sizeof(int);
    if (need > g->scratch_bytes) {
        std::ostringstream m;
        m << "rt_step_noalloc: this grid's step writes partial sums of " << nb << " blocks ("
          << need << " bytes), more than the static scratch holds (" << g->scratch_bytes
          << " bytes); use rt_step";
        return fail(RT_EINVAL, m.str());
    }
    unsigned char *base = static_cast<unsigned char *>(g->scratch);
    const rt::Partials P{reinterpret_cast<double *>(base), reinterpret_cast<int *>(base + off)};
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    int rc = rt::launch_step(g, (hipStream_t)stream, I_in, I_out, T, rho, u_tet, kappa_a, kappa_s,
                             dt, dT0, lum, I_star, P);
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc != RT_OK) return fail(rc, "kernel launch failed");
    return RT_OK;
}

int rt_step_adjoint(rt_grid *g, void *stream, const void *I_n, const double *T_n,
                    const double *rho, const double *u_tet, const double *kappa_a,
                    const double *kappa_s, double dt, double lum_weight, const void *lamI_np1,
                    const double *lamT_np1, void *lamI_n, double *lamT_n, void *work,
                    double *grad_kappa_a, double *grad_kappa_s, const void *I_star) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (!I_n || !T_n || !rho || !u_tet || !kappa_a || !kappa_s || !lamI_np1 || !lamT_np1 ||
        !lamI_n || !lamT_n || !work)
        return fail(RT_EINVAL, "NULL state pointer");
    if (work == I_n || work == lamI_np1 || work == lamI_n || lamI_n == I_n)
        return fail(RT_EINVAL, "work must not alias the state or the adjoint buffers");
    if (I_star && (I_star == work || I_star == lamI_n))
        return fail(RT_EINVAL, "I_star must not alias work or lamI_n");
    if (g->integrator == 2 || g->dg.tau_coeff > 0.0 || g->dg.rad_velocity || g->dg.ang_recon)
        return fail(RT_EINVAL, "the adjoint covers the one-stage step without the optical-depth-aware "
                               "flux, the velocity substitute and angular PLM");
    if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(lum_weight))
        return fail(RT_EINVAL, "dt must be positive and finite");
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    int rc = rt::launch_adjoint(g, (hipStream_t)stream, I_n, T_n, rho, u_tet, kappa_a, kappa_s, dt,
                                lum_weight, lamI_np1, lamT_np1, lamI_n, lamT_n, work, grad_kappa_a,
                                grad_kappa_s, I_star);
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc != RT_OK) return fail(rc, "kernel launch failed");
    return RT_OK;
}

int rt_moments(rt_grid *g, void *stream, const void *I, const double *u_tet, double *R_tet,
               double *R0_cov, double *E_fluid) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (!I || (E_fluid && !u_tet)) return fail(RT_EINVAL, "NULL input pointer");
    if (!R_tet && !R0_cov && !E_fluid) return RT_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    int rc = rt::launch_moments(g, (hipStream_t)stream, I, u_tet, R_tet, R0_cov, E_fluid);
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc != RT_OK) return fail(rc, "kernel launch failed");
    return RT_OK;
}

int rt_gas_update(rt_grid *g, void *stream, const double *dT0, const double *T_pre,
                  double *rho, double *u_tet, double *T, int32_t *status) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    if (!dT0 || !T_pre || !rho || !u_tet || !T) return fail(RT_EINVAL, "NULL state pointer");
    if ((const void *)dT0 == (const void *)rho || (const void *)dT0 == (const void *)u_tet ||
        (const void *)dT0 == (const void *)T || (const void *)T_pre == (const void *)rho ||
        (const void *)T_pre == (const void *)u_tet)
        return fail(RT_EINVAL, "dT0 and T_pre must not alias the gas state (T_pre may alias T)");
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    int rc = rt::launch_gas_update(g, (hipStream_t)stream, dT0, T_pre, rho, u_tet, T, status);
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc != RT_OK) return fail(rc, "kernel launch failed");
    return RT_OK;
}

int rt_stats(rt_grid *g, int64_t *no_root_events, double *masked_energy) {
    if (!g) return fail(RT_EINVAL, "grid is NULL");
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    long long nr = 0;
    double me = 0.0;
    hipError_t e1 = hipDeviceSynchronize();
    hipError_t e2 = hipMemcpy(&nr, g->noroot, sizeof(nr), hipMemcpyDeviceToHost);
    hipError_t e3 = hipMemcpy(&me, g->ledger, sizeof(me), hipMemcpyDeviceToHost);
    (void)hipSetDevice(cur);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return fail(RT_EDEVICE, "reading statistics failed");
    if (no_root_events) *no_root_events = nr;
    if (masked_energy) *masked_energy = me;
    return RT_OK;
}

void rt_free(rt_grid *g) {
    if (!g) return;
    release(g);
    delete g;
}

}  // extern "C"
