// Latitude-longitude angular grid (paper Sec. 2.6): n_zeta + 1 circles of
// latitude equally spaced in cos(zeta) between the poles on the tetrad x^3
// axis, n_psi + 1 meridians equally spaced in psi from the x^1 axis, so all
// n_zeta n_psi cells subtend the same solid angle.  Edges are the arcs
// between neighbouring cells: along a circle of latitude (normal +zeta-hat,
// length sin(zeta) dpsi) or along a meridian (normal +psi-hat, length dzeta).
// For angular PLM (Sec. 2.3) every edge also records the next cell beyond
// each end along its own coordinate line; across a pole that is the cell of
// the same row at psi + pi.
#include <cmath>
#include <stdexcept>

#include "rt_host.h"

namespace rt {

Geodesic build_latlong(int nz, int np) {
    if (nz < 2 || np < 2 || (np & 1)) throw std::runtime_error("latitude-longitude grid: bad size");
    const double two_pi = 2.0 * M_PI;
    const double dpsi = two_pi / np;
    std::vector<double> cb(nz + 1), zb(nz + 1);
    for (int l = 0; l <= nz; ++l) {
        cb[l] = l == nz ? -1.0 : 1.0 - 2.0 * (double)l / nz;
        zb[l] = std::acos(cb[l]);
    }
    Geodesic g;
    g.nlev = 0;
    g.nang = nz * np;
    g.nhat.resize(3 * g.nang);
    g.domega.resize(g.nang);
    auto id = [np](int l, int m) { return l * np + ((m % np) + np) % np; };
    for (int l = 0; l < nz; ++l) {
        const double z = std::acos(0.5 * (cb[l] + cb[l + 1]));
        for (int m = 0; m < np; ++m) {
            const double p = dpsi * (m + 0.5);
            const int n = id(l, m);
            g.nhat[3 * n] = std::sin(z) * std::cos(p);
            g.nhat[3 * n + 1] = std::sin(z) * std::sin(p);
            g.nhat[3 * n + 2] = std::cos(z);
            g.domega[n] = (cb[l] - cb[l + 1]) * dpsi;
        }
    }
    g.nedge = (nz - 1) * np + nz * np;
    g.lo.resize(g.nedge);
    g.hi.resize(g.nedge);
    g.ll.resize(g.nedge);
    g.rr.resize(g.nedge);
    g.len.resize(g.nedge);
    g.mid.resize(3 * g.nedge);
    g.nu.resize(3 * g.nedge);
    int e = 0;
    auto put = [&](int lo, int hi, int ll, int rr, double len, double mz, double mp, const double nu[3]) {
        g.lo[e] = lo;
        g.hi[e] = hi;
        g.ll[e] = ll;
        g.rr[e] = rr;
        g.len[e] = len;
        g.mid[3 * e] = std::sin(mz) * std::cos(mp);
        g.mid[3 * e + 1] = std::sin(mz) * std::sin(mp);
        g.mid[3 * e + 2] = std::cos(mz);
        for (int c = 0; c < 3; ++c) g.nu[3 * e + c] = nu[c];
        ++e;
    };
    // circles of latitude between rows l and l + 1
    for (int l = 0; l + 1 < nz; ++l) {
        const double z = zb[l + 1];
        for (int m = 0; m < np; ++m) {
            const double p = dpsi * (m + 0.5);
            const double nu[3] = {std::cos(z) * std::cos(p), std::cos(z) * std::sin(p), -std::sin(z)};
            const int ll = l > 0 ? id(l - 1, m) : id(0, m + np / 2);
            const int rr = l + 2 < nz ? id(l + 2, m) : id(nz - 1, m + np / 2);
            put(id(l, m), id(l + 1, m), ll, rr, std::sin(z) * dpsi, z, p, nu);
        }
    }
    // meridians between columns m and m + 1
    for (int l = 0; l < nz; ++l) {
        const double zm = 0.5 * (zb[l] + zb[l + 1]);
        for (int m = 0; m < np; ++m) {
            const double p = dpsi * (m + 1);
            const double nu[3] = {-std::sin(p), std::cos(p), 0.0};
            put(id(l, m), id(l, m + 1), id(l, m - 1), id(l, m + 2), zb[l + 1] - zb[l], zm, p, nu);
        }
    }
    g.adj_e.assign(kMaxNbr * g.nang, -1);
    g.adj_s.assign(kMaxNbr * g.nang, 0);
    std::vector<int> deg(g.nang, 0);
    for (int k = 0; k < g.nedge; ++k) {
        const int lo = g.lo[k], hi = g.hi[k];
        if (deg[lo] >= kMaxNbr || deg[hi] >= kMaxNbr)
            throw std::runtime_error("latitude-longitude grid: more than 6 edges");
        g.adj_e[kMaxNbr * lo + deg[lo]] = k;
        g.adj_s[kMaxNbr * lo + deg[lo]++] = +1;
        g.adj_e[kMaxNbr * hi + deg[hi]] = k;
        g.adj_s[kMaxNbr * hi + deg[hi]++] = -1;
    }
    return g;
}

}  // namespace rt
