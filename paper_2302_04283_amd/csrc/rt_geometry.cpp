// Host FP64 geometry precompute (paper Sec. 2.1-2.2, 2.4, 2.6).
//
// From the metric g_{mu nu}, the tetrad e^mu_{b^} and their spatial
// derivatives at each geometry cell (stationary: d_0 = 0):
//   Gamma^m_{nl}   = 1/2 g^{ms} (d_n g_{sl} + d_l g_{sn} - d_s g_{nl})
//   omega^c_{ab}   = e^c_m e^d_b (d_d e^m_a + Gamma^m_{dl} e^l_a)      (Sec. 2.2)
//   n^mu           = e^mu_{b^} n^{b^},  n^{b^} = (1, n^)                 (Sec. 2.2)
//   n_0            = g_{0 mu} n^mu
// and the coefficients the step consumes:
//   q      = n^0 n_0                       conserved / primitive factor
//   C      = dA n^a n_0 (face centre)      spatial flux coefficient (Sec. 2.4)
//   v, w   = L_e W(m_e).nu_e, v n_0(m_e)   angular flux on edge e, with
//            W(m) = -omega^i(m,m) + m^i omega^0(m,m), the tetrad-frame
//            direction velocity on the sphere (the paper's n^zeta, n^psi)
//   mask   = |n_0| < n0_crit               (Sec. 2.4)
#include <cmath>
#include <cstring>
#include <sstream>

#include "rt_host.h"

namespace rt {
namespace {

bool invert4(const double *a, double *out) {
    double m[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? a[4 * i + j] : (j - 4 == i ? 1.0 : 0.0);
    for (int c = 0; c < 4; ++c) {
        int p = c;
        for (int r = c + 1; r < 4; ++r)
            if (std::fabs(m[r][c]) > std::fabs(m[p][c])) p = r;
        if (m[p][c] == 0.0) return false;
        if (p != c)
            for (int j = 0; j < 8; ++j) std::swap(m[p][j], m[c][j]);
        double inv = 1.0 / m[c][c];
        for (int j = 0; j < 8; ++j) m[c][j] *= inv;
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            double f = m[r][c];
            if (f != 0.0)
                for (int j = 0; j < 8; ++j) m[r][j] -= f * m[c][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) out[4 * i + j] = m[i][j + 4];
    return true;
}

const double kEta[4] = {-1.0, 1.0, 1.0, 1.0};

// omega[c][a][b] at one point.  g[16], dg[3][16] (d/dx^1..3), e[16] = e^mu_b
// stored [mu][b], de[3][16].
void ricci_rotation(const double *g, const double *dg3, const double *e, const double *de3,
                    const double *ginv, double *om) {
    double dg[4][16] = {};
    double de[4][16] = {};
    for (int d = 1; d < 4; ++d) {
        std::memcpy(dg[d], dg3 + 16 * (d - 1), 16 * sizeof(double));
        std::memcpy(de[d], de3 + 16 * (d - 1), 16 * sizeof(double));
    }
    double Gam[4][4][4];
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n)
            for (int l = 0; l < 4; ++l) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k)
                    s += ginv[4 * m + k] * (dg[n][4 * k + l] + dg[l][4 * k + n] - dg[k][4 * n + l]);
                Gam[m][n][l] = 0.5 * s;
            }
    // nab[d][m][a] = d_d e^m_a + Gamma^m_{d l} e^l_a
    double nab[4][4][4];
    for (int d = 0; d < 4; ++d)
        for (int m = 0; m < 4; ++m)
            for (int a = 0; a < 4; ++a) {
                double s = de[d][4 * m + a];
                for (int l = 0; l < 4; ++l) s += Gam[m][d][l] * e[4 * l + a];
                nab[d][m][a] = s;
            }
    // einv[c][m] = eta^{cc} g_{m n} e^n_c
    double einv[4][4];
    for (int c = 0; c < 4; ++c)
        for (int m = 0; m < 4; ++m) {
            double s = 0.0;
            for (int n = 0; n < 4; ++n) s += g[4 * m + n] * e[4 * n + c];
            einv[c][m] = kEta[c] * s;
        }
    for (int c = 0; c < 4; ++c)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double s = 0.0;
                for (int m = 0; m < 4; ++m)
                    for (int d = 0; d < 4; ++d) s += einv[c][m] * e[4 * d + b] * nab[d][m][a];
                om[16 * c + 4 * a + b] = s;
            }
}

void dir_up(const double *e, const double *nh, double *nu) {
    for (int m = 0; m < 4; ++m)
        nu[m] = e[4 * m] + e[4 * m + 1] * nh[0] + e[4 * m + 2] * nh[1] + e[4 * m + 3] * nh[2];
}

double n0_low(const double *g, const double *nu) {
    return g[0] * nu[0] + g[1] * nu[1] + g[2] * nu[2] + g[3] * nu[3];
}

}  // namespace

int build_tables(const rt_grid_desc &d, const Geodesic &ang, HostTables &t, std::string &err) {
    const int g0 = d.geo_extent[0], g1 = d.geo_extent[1], g2 = d.geo_extent[2];
    const int G = g0 * g1 * g2;
    const int N = ang.nang, E = ang.nedge;
    t.G = G;
    t.q.assign((size_t)G * N, 0.0);
    t.mask.assign((size_t)G * N, 0);
    t.vw.assign((size_t)G * E * 2, 0.0);
    t.n0u.assign(G, 0.0);
    t.E0.assign((size_t)G * 16, 0.0);
    t.gas_map.assign((size_t)G * 16, 0.0);
    t.vol.assign(d.vol, d.vol + G);
    t.has_edges = false;
    t.masked_count = 0;
    for (int c = 0; c < G; ++c) {
        const double *g = d.gcov_c + 16 * c;
        const double *e = d.tet_c + 16 * c;
        double ginv[16];
        if (!invert4(g, ginv)) {
            err = "singular metric at a cell centre";
            return RT_EGEOM;
        }
        // orthonormal tetrad, normal-observer time leg (Sec. 2.1)
        double worst = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double s = 0.0;
                for (int m = 0; m < 4; ++m)
                    for (int n = 0; n < 4; ++n) s += g[4 * m + n] * e[4 * m + a] * e[4 * n + b];
                worst = std::fmax(worst, std::fabs(s - (a == b ? kEta[a] : 0.0)));
            }
        if (worst > 1e-10) {
            std::ostringstream os;
            os << "tetrad not orthonormal at geometry cell " << c << " (|g e e - eta| = " << worst << ")";
            err = os.str();
            return RT_EGEOM;
        }
        if (!(-ginv[0] > 0.0)) {
            err = "g^{00} must be negative";
            return RT_EGEOM;
        }
        double alpha = 1.0 / std::sqrt(-ginv[0]);
        for (int m = 0; m < 4; ++m)
            if (std::fabs(e[4 * m] + alpha * ginv[m]) > 1e-10 * (1.0 + std::fabs(alpha * ginv[m]))) {
                err = "tetrad time leg is not the normal observer -alpha g^{0mu}";
                return RT_EGEOM;
            }
        t.n0u[c] = e[0];
        // normal-observer tetrad: e^{0^}_mu = (alpha, 0, 0, 0) and
        // e^{b^}_mu g^{mu nu} = eta^{b b} e^nu_{b^}, so the tetrad row of a
        // stress tensor is T^{0^ b^} = alpha eta^{bb} e^nu_{b^} T^0_nu
        for (int b = 0; b < 4; ++b)
            for (int m = 0; m < 4; ++m)
                t.gas_map[16 * c + 4 * b + m] = (1.0 / e[0]) * kEta[b] * e[4 * m + b];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double s = 0.0;
                for (int m = 0; m < 4; ++m) s += g[4 * a + m] * e[4 * m + b];
                t.E0[16 * c + 4 * a + b] = s;
            }
        for (int n = 0; n < N; ++n) {
            double nu[4];
            dir_up(e, &ang.nhat[3 * n], nu);
            double nl0 = n0_low(g, nu);
            t.q[(size_t)c * N + n] = nu[0] * nl0;
            if (std::fabs(nl0) < d.n0_crit) {
                t.mask[(size_t)c * N + n] = 1;
                ++t.masked_count;
            }
        }
        double om[64];
        ricci_rotation(g, d.dgcov_c + 48 * c, e, d.dtet_c + 48 * c, ginv, om);
        for (int k = 0; k < E; ++k) {
            const double *m = &ang.mid[3 * k];
            const double m4[4] = {1.0, m[0], m[1], m[2]};
            double qq[4];
            for (int cc = 0; cc < 4; ++cc) {
                double s = 0.0;
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) s += om[16 * cc + 4 * a + b] * m4[a] * m4[b];
                qq[cc] = s;
            }
            double Wn = 0.0;
            for (int i = 0; i < 3; ++i) Wn += (-qq[i + 1] + m[i] * qq[0]) * ang.nu[3 * k + i];
            double v = ang.len[k] * Wn;
            double nu[4];
            dir_up(e, m, nu);
            t.vw[((size_t)c * E + k) * 2] = v;
            t.vw[((size_t)c * E + k) * 2 + 1] = v * n0_low(g, nu);
            if (v != 0.0) t.has_edges = true;
        }
    }
    // faces
    for (int a = 0; a < 3; ++a) {
        int fe[3];
        for (int b = 0; b < 3; ++b)
            fe[b] = (b == a) ? (d.geo_extent[b] > 1 ? d.n[b] + 1 : 1) : d.geo_extent[b];
        const int F = fe[0] * fe[1] * fe[2];
        t.F[a] = F;
        t.C[a].assign((size_t)F * N, 0.0);
        t.sgn[a].assign((size_t)F * N, 0);
        for (int f = 0; f < F; ++f) {
            const double *g = d.gcov_f[a] + 16 * f;
            const double *e = d.tet_f[a] + 16 * f;
            const double A = d.area[a][f];
            for (int n = 0; n < N; ++n) {
                double nu[4];
                dir_up(e, &ang.nhat[3 * n], nu);
                double na = nu[a + 1];
                t.C[a][(size_t)f * N + n] = A * na * n0_low(g, nu);
                t.sgn[a][(size_t)f * N + n] = na > 0.0 ? 1 : (na < 0.0 ? -1 : 0);
            }
        }
    }
    return RT_OK;
}

}  // namespace rt
