// Test harness: the library's host-only code (descriptor checks, angular
// grids, MAPR tables, FP64 geometry tables) behind two C entry points, so
// a test can build it with AddressSanitizer/UndefinedBehaviorSanitizer and
// drive it from Python with the same descriptors rt_init_grid receives.
// Besides running the code under the sanitizers it checks the table sizes
// and index ranges the device kernels rely on.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>

#include "rt_host.h"

namespace {

void put_err(const std::string &e, char *err, int errlen) {
    if (!err || errlen <= 0) return;
    std::snprintf(err, (size_t)errlen, "%s", e.c_str());
}

// index tables of an angular grid within range, weights summing to 4 pi
std::string check_angles(const rt::Geodesic &a) {
    const int N = a.nang, E = a.nedge;
    if ((int)a.nhat.size() != 3 * N || (int)a.domega.size() != N) return "angle table sizes";
    if ((int)a.lo.size() != E || (int)a.hi.size() != E) return "edge table sizes";
    if ((int)a.adj_e.size() != rt::kMaxNbr * N || (int)a.adj_s.size() != rt::kMaxNbr * N)
        return "adjacency table sizes";
    double sum = 0.0;
    for (int n = 0; n < N; ++n) sum += a.domega[n];
    if (std::fabs(sum - 4.0 * M_PI) > 1e-12) return "solid angles do not sum to 4 pi";
    for (int e = 0; e < E; ++e)
        if (a.lo[e] < 0 || a.lo[e] >= N || a.hi[e] < 0 || a.hi[e] >= N || a.lo[e] == a.hi[e])
            return "edge endpoint out of range";
    for (int i = 0; i < rt::kMaxNbr * N; ++i) {
        const int e = a.adj_e[i];
        if (e < -1 || e >= E) return "adjacent edge out of range";
        if (e >= 0) {
            const int n = i / rt::kMaxNbr;
            const int self = a.adj_s[i] > 0 ? a.lo[e] : a.hi[e];
            if (self != n) return "adjacency does not name the direction";
        }
    }
    // the edge records pack the edge and the other direction in 15 bits each
    if (E >= (1 << 15) || N >= (1 << 15)) return "edge record overflow";
    return "";
}

}  // namespace

extern "C" {

// Builds everything rt_init_grid builds on the host for descriptor d:
// RT_OK, or the error code with its reason in err.
int rt_host_check(const rt_grid_desc *d, char *err, int errlen) {
    std::string e;
    try {
        int rc = rt::check_desc(d, e);
        if (rc != RT_OK) {
            put_err(e, err, errlen);
            return rc;
        }
        const rt::Geodesic ang =
            d->n_zeta > 0 ? rt::build_latlong(d->n_zeta, d->n_psi) : rt::build_geodesic(d->nlev);
        e = check_angles(ang);
        if (!e.empty()) {
            put_err(e, err, errlen);
            return RT_EGEOM;
        }
        rt::HostTables t;
        rc = rt::build_tables(*d, ang, t, e);
        if (rc != RT_OK) {
            put_err(e, err, errlen);
            return rc;
        }
        const size_t G = (size_t)t.G, N = (size_t)ang.nang;
        if (t.q.size() != G * N || t.mask.size() != G * N || t.n0u.size() != G ||
            t.E0.size() != 16 * G || t.gas_map.size() != 16 * G || t.vol.size() != G)
            e = "cell table sizes";
        for (int a = 0; a < 3 && e.empty(); ++a)
            if (t.C[a].size() != (size_t)t.F[a] * N || t.sgn[a].size() != (size_t)t.F[a] * N)
                e = "face table sizes";
        if (e.empty() && t.has_edges && t.vw.size() != G * ang.nedge * 2) e = "edge weight sizes";
        if (e.empty() && d->ang_recon == 2) {
            std::vector<int> nb;
            std::vector<double> inv, dd;
            std::vector<int8_t> cnt;
            rt::build_mapr(ang, nb, inv, cnt, dd);
            if (nb.size() != N * rt::kMaxNbr || cnt.size() != N || inv.size() != N * rt::kMaxNbr * 4 ||
                dd.size() != (size_t)ang.nedge * 4)
                e = "MAPR table sizes";
            for (size_t i = 0; i < nb.size() && e.empty(); ++i)
                if (nb[i] < 0 || nb[i] >= (int)N) e = "MAPR neighbour out of range";
        }
        if (!e.empty()) {
            put_err(e, err, errlen);
            return RT_EGEOM;
        }
    } catch (const std::exception &ex) {
        put_err(ex.what(), err, errlen);
        return RT_EINVAL;
    }
    put_err("", err, errlen);
    return RT_OK;
}

// The angular grid alone: geodesic (nlev > 0) or latitude-longitude.
int rt_host_angles(int nlev, int n_zeta, int n_psi, char *err, int errlen) {
    try {
        const rt::Geodesic a = nlev > 0 ? rt::build_geodesic(nlev) : rt::build_latlong(n_zeta, n_psi);
        const std::string e = check_angles(a);
        put_err(e, err, errlen);
        return e.empty() ? RT_OK : RT_EGEOM;
    } catch (const std::exception &ex) {
        put_err(ex.what(), err, errlen);
        return RT_EINVAL;
    }
}

}  // extern "C"
