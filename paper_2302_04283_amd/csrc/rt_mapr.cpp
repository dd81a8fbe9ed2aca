// Host tables of minimum-angle plane reconstruction (MAPR) on the geodesic
// grid (paper Sec. 2.6, after Christov & Popov's method as used on hexagonal
// geodesic grids by Florinski et al.).  Each direction cell is seen in the
// plane tangent to the sphere at its centre (gnomonic coordinates); its
// neighbours are taken in angular order, and each pair of consecutive
// neighbours defines a candidate plane through the cell's value whose
// gradient g solves [x_i; x_{i+1}] g = [I_i - I_c; I_{i+1} - I_c].  The
// kernel keeps the candidate of smallest |g| (the plane closest to
// horizontal) and evaluates I_c + g . d at each edge midpoint d.
#include <cmath>
#include <stdexcept>

#include "rt_host.h"

namespace rt {
namespace {

struct Basis {
    double v[3], a[3], b[3];
};

Basis tangent_basis(const double *v) {
    // first axis: the projection of +z (or of +x near the poles)
    Basis B;
    for (int c = 0; c < 3; ++c) B.v[c] = v[c];
    const double ref[3] = {std::fabs(v[2]) < 0.9 ? 0.0 : 1.0, 0.0, std::fabs(v[2]) < 0.9 ? 1.0 : 0.0};
    const double r = ref[0] * v[0] + ref[1] * v[1] + ref[2] * v[2];
    double n = 0.0;
    for (int c = 0; c < 3; ++c) {
        B.a[c] = ref[c] - r * v[c];
        n += B.a[c] * B.a[c];
    }
    n = std::sqrt(n);
    for (int c = 0; c < 3; ++c) B.a[c] /= n;
    B.b[0] = v[1] * B.a[2] - v[2] * B.a[1];
    B.b[1] = v[2] * B.a[0] - v[0] * B.a[2];
    B.b[2] = v[0] * B.a[1] - v[1] * B.a[0];
    return B;
}

void project(const Basis &B, const double *p, double &x, double &y) {
    const double s = p[0] * B.v[0] + p[1] * B.v[1] + p[2] * B.v[2];
    x = (p[0] * B.a[0] + p[1] * B.a[1] + p[2] * B.a[2]) / s;
    y = (p[0] * B.b[0] + p[1] * B.b[1] + p[2] * B.b[2]) / s;
}

}  // namespace

void build_mapr(const Geodesic &g, std::vector<int> &nb, std::vector<double> &inv,
                std::vector<int8_t> &cnt, std::vector<double> &d) {
    const int N = g.nang, E = g.nedge;
    nb.assign((size_t)N * kMaxNbr, 0);
    inv.assign((size_t)N * kMaxNbr * 4, 0.0);
    cnt.assign(N, 0);
    d.assign((size_t)E * 4, 0.0);
    std::vector<Basis> basis(N);
    for (int n = 0; n < N; ++n) {
        basis[n] = tangent_basis(&g.nhat[3 * n]);
        int k = 0;
        int ids[kMaxNbr];
        double ang[kMaxNbr], px[kMaxNbr], py[kMaxNbr];
        for (int s = 0; s < kMaxNbr; ++s) {
            const int e = g.adj_e[n * kMaxNbr + s];
            if (e < 0) break;
            const int m = g.lo[e] == n ? g.hi[e] : g.lo[e];
            ids[k] = m;
            project(basis[n], &g.nhat[3 * m], px[k], py[k]);
            ang[k] = std::atan2(py[k], px[k]);
            ++k;
        }
        if (k < 3) throw std::runtime_error("MAPR needs at least three neighbours");
        // insertion sort by angle (counter-clockwise about the outward
        // direction), then rotate to start at the smallest neighbour index:
        // the order breaks ties between equally flat planes and must not
        // depend on the tangent basis
        for (int i = 1; i < k; ++i)
            for (int j = i; j > 0 && ang[j] < ang[j - 1]; --j) {
                std::swap(ang[j], ang[j - 1]);
                std::swap(ids[j], ids[j - 1]);
                std::swap(px[j], px[j - 1]);
                std::swap(py[j], py[j - 1]);
            }
        int first = 0;
        for (int i = 1; i < k; ++i)
            if (ids[i] < ids[first]) first = i;
        int rid[kMaxNbr];
        double rx[kMaxNbr], ry[kMaxNbr];
        for (int i = 0; i < k; ++i) {
            rid[i] = ids[(first + i) % k];
            rx[i] = px[(first + i) % k];
            ry[i] = py[(first + i) % k];
        }
        for (int i = 0; i < k; ++i) {
            ids[i] = rid[i];
            px[i] = rx[i];
            py[i] = ry[i];
        }
        cnt[n] = (int8_t)k;
        for (int i = 0; i < kMaxNbr; ++i) nb[(size_t)n * kMaxNbr + i] = i < k ? ids[i] : n;
        for (int i = 0; i < k; ++i) {
            const int j = (i + 1) % k;
            const double det = px[i] * py[j] - py[i] * px[j];
            if (!(std::fabs(det) > 0.0)) throw std::runtime_error("MAPR: collinear neighbours");
            double *M = &inv[((size_t)n * kMaxNbr + i) * 4];
            M[0] = py[j] / det;     // g_x = M0 dI_i + M1 dI_j
            M[1] = -py[i] / det;
            M[2] = -px[j] / det;    // g_y = M2 dI_i + M3 dI_j
            M[3] = px[i] / det;
        }
    }
    for (int e = 0; e < E; ++e) {
        project(basis[g.lo[e]], &g.mid[3 * e], d[4 * e], d[4 * e + 1]);
        project(basis[g.hi[e]], &g.mid[3 * e], d[4 * e + 2], d[4 * e + 3]);
    }
}

}  // namespace rt
