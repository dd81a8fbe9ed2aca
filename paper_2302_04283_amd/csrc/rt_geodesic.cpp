// Geodesic angular grid (paper Sec. 2.6): the icosahedron's 20 faces are cut
// into N^2 flat triangles; the projected triangulation vertices are the
// direction cells and the projected centres of the flat triangles are the
// corners of the pentagonal/hexagonal cells, joined by great-circle arcs.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <stdexcept>
#include <utility>

#include "rt_host.h"

namespace rt {
namespace {

using V3 = std::array<double, 3>;

V3 operator+(const V3 &a, const V3 &b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
V3 operator-(const V3 &a, const V3 &b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
V3 operator*(double s, const V3 &a) { return {s * a[0], s * a[1], s * a[2]}; }
double dot(const V3 &a, const V3 &b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
V3 cross(const V3 &a, const V3 &b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double norm(const V3 &a) { return std::sqrt(dot(a, a)); }
V3 unit(const V3 &a) { return (1.0 / norm(a)) * a; }

// Solid angle of the spherical triangle (a, b, c) of unit vectors,
// Van Oosterom & Strackee (1983).
double tri_solid_angle(const V3 &a, const V3 &b, const V3 &c) {
    double num = std::fabs(dot(a, cross(b, c)));
    double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
    return 2.0 * std::atan2(num, den);
}

}  // namespace

Geodesic build_geodesic(int N) {
    if (N < 1) throw std::invalid_argument("nlev must be >= 1");
    const double pi = 3.14159265358979323846;
    // icosahedron: 0 = +z pole, 1..5 upper ring (azimuth 72k deg), 6..10 lower
    // ring (72k + 36 deg), 11 = -z pole; vertex 1 lies in the x-z plane, x > 0.
    std::vector<V3> ico(12);
    const double zr = 1.0 / std::sqrt(5.0), rr = 2.0 / std::sqrt(5.0);
    ico[0] = {0.0, 0.0, 1.0};
    ico[11] = {0.0, 0.0, -1.0};
    for (int k = 0; k < 5; ++k) {
        double pu = 2.0 * pi * k / 5.0, pl = 2.0 * pi * (k + 0.5) / 5.0;
        ico[1 + k] = {rr * std::cos(pu), rr * std::sin(pu), zr};
        ico[6 + k] = {rr * std::cos(pl), rr * std::sin(pl), -zr};
    }
    std::vector<std::array<int, 3>> faces;
    for (int k = 0; k < 5; ++k) {
        int u0 = 1 + k, u1 = 1 + (k + 1) % 5, l0 = 6 + k, l1 = 6 + (k + 1) % 5;
        faces.push_back({0, u0, u1});
        faces.push_back({u0, l0, u1});
        faces.push_back({u1, l0, l1});
        faces.push_back({11, l1, l0});
    }

    // flat triangulation points (barycentric), their cell, and flat triangles
    std::vector<V3> flat;              // flat point positions
    std::vector<int> on_edge;          // lies on an icosahedron edge
    std::vector<std::array<int, 3>> tri;
    for (const auto &f : faces) {
        const V3 &A = ico[f[0]], &B = ico[f[1]], &C = ico[f[2]];
        std::vector<int> id((N + 1) * (N + 1), -1);
        for (int i = 0; i <= N; ++i)
            for (int j = 0; i + j <= N; ++j) {
                int k = N - i - j;
                V3 p = (1.0 / N) * ((double)k * A + (double)i * B + (double)j * C);
                id[i * (N + 1) + j] = (int)flat.size();
                flat.push_back(p);
                on_edge.push_back(i == 0 || j == 0 || k == 0);
            }
        auto P = [&](int i, int j) { return id[i * (N + 1) + j]; };
        for (int i = 0; i < N; ++i)
            for (int j = 0; i + j < N; ++j) {
                tri.push_back({P(i, j), P(i + 1, j), P(i, j + 1)});
                if (i + j + 2 <= N) tri.push_back({P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)});
            }
    }
    // merge the copies of points shared by neighbouring faces
    std::vector<int> cell_of(flat.size(), -1);
    std::vector<V3> cdir;
    std::vector<int> edge_reps;        // representative flat index of edge cells
    for (size_t p = 0; p < flat.size(); ++p) {
        V3 u = unit(flat[p]);
        if (on_edge[p]) {
            for (int r : edge_reps) {
                if (norm(unit(flat[r]) - u) < 1e-9) {
                    cell_of[p] = cell_of[r];
                    break;
                }
            }
            if (cell_of[p] < 0) edge_reps.push_back((int)p);
        }
        if (cell_of[p] < 0) {
            cell_of[p] = (int)cdir.size();
            cdir.push_back(u);
        }
    }
    const int nang = (int)cdir.size();
    if (nang != 10 * N * N + 2) throw std::runtime_error("geodesic grid: wrong cell count");

    // canonical order: rings of equal polar angle, each by azimuth from -0.01 rad
    std::vector<double> zeta(nang), psi(nang);
    for (int c = 0; c < nang; ++c) {
        const V3 &v = cdir[c];
        zeta[c] = std::atan2(std::hypot(v[0], v[1]), v[2]);
        double ps = std::atan2(v[1], v[0]) + 0.01;
        ps = std::fmod(ps + 2.0 * pi, 2.0 * pi);
        psi[c] = ps;
    }
    std::vector<int> byz(nang);
    for (int c = 0; c < nang; ++c) byz[c] = c;
    std::stable_sort(byz.begin(), byz.end(), [&](int a, int b) { return zeta[a] < zeta[b]; });
    std::vector<int> ring(nang, 0);
    for (int k = 1; k < nang; ++k)
        ring[byz[k]] = ring[byz[k - 1]] + (zeta[byz[k]] - zeta[byz[k - 1]] > 1e-9 ? 1 : 0);
    std::vector<int> order(nang);
    for (int c = 0; c < nang; ++c) order[c] = c;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (ring[a] != ring[b]) return ring[a] < ring[b];
        return psi[a] < psi[b];
    });
    std::vector<int> rank(nang);
    for (int r = 0; r < nang; ++r) rank[order[r]] = r;

    Geodesic g;
    g.nlev = N;
    g.nang = nang;
    g.nhat.resize(3 * nang);
    for (int r = 0; r < nang; ++r)
        for (int c = 0; c < 3; ++c) g.nhat[3 * r + c] = cdir[order[r]][c];

    // triangles as canonical cell triples, and their projected centres
    const int T = (int)tri.size();
    std::vector<std::array<int, 3>> tc(T);
    std::vector<V3> corner(T);
    for (int t = 0; t < T; ++t) {
        V3 s = {0, 0, 0};
        for (int k = 0; k < 3; ++k) {
            tc[t][k] = rank[cell_of[tri[t][k]]];
            s = s + flat[tri[t][k]];
        }
        corner[t] = unit((1.0 / 3.0) * s);
    }

    // polygon areas: fan of spherical triangles around the cell direction
    std::vector<std::vector<int>> inc(nang);
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < 3; ++k) inc[tc[t][k]].push_back(t);
    g.domega.assign(nang, 0.0);
    for (int c = 0; c < nang; ++c) {
        V3 v = {g.nhat[3 * c], g.nhat[3 * c + 1], g.nhat[3 * c + 2]};
        V3 ref = std::fabs(v[2]) < 0.9 ? V3{0.0, 0.0, 1.0} : V3{1.0, 0.0, 0.0};
        V3 t1 = unit(ref - dot(ref, v) * v);
        V3 t2 = cross(v, t1);
        std::vector<std::pair<double, int>> ang;
        for (int t : inc[c]) ang.push_back({std::atan2(dot(corner[t], t2), dot(corner[t], t1)), t});
        std::sort(ang.begin(), ang.end());
        double s = 0.0;
        const int k = (int)ang.size();
        for (int m = 0; m < k; ++m)
            s += tri_solid_angle(v, corner[ang[m].second], corner[ang[(m + 1) % k].second]);
        g.domega[c] = s;
    }

    // edges: one per pair of cells sharing a triangulation edge
    std::map<std::pair<int, int>, std::vector<int>> share;
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < 3; ++k) {
            int a = tc[t][k], b = tc[t][(k + 1) % 3];
            share[{std::min(a, b), std::max(a, b)}].push_back(t);
        }
    g.nedge = (int)share.size();
    g.lo.resize(g.nedge);
    g.hi.resize(g.nedge);
    g.len.resize(g.nedge);
    g.mid.resize(3 * g.nedge);
    g.nu.resize(3 * g.nedge);
    g.adj_e.assign(kMaxNbr * nang, -1);
    g.adj_s.assign(kMaxNbr * nang, 0);
    std::vector<int> deg(nang, 0);
    int e = 0;
    for (const auto &kv : share) {
        if (kv.second.size() != 2) throw std::runtime_error("geodesic grid: open edge");
        const V3 &p1 = corner[kv.second[0]], &p2 = corner[kv.second[1]];
        int lo = kv.first.first, hi = kv.first.second;
        V3 cr = cross(p1, p2);
        V3 m = unit(p1 + p2);
        V3 n = unit(cr);
        V3 dlh = {g.nhat[3 * hi] - g.nhat[3 * lo], g.nhat[3 * hi + 1] - g.nhat[3 * lo + 1],
                  g.nhat[3 * hi + 2] - g.nhat[3 * lo + 2]};
        if (dot(n, dlh) < 0.0) n = -1.0 * n;
        g.lo[e] = lo;
        g.hi[e] = hi;
        g.len[e] = std::atan2(norm(cr), dot(p1, p2));
        for (int c = 0; c < 3; ++c) {
            g.mid[3 * e + c] = m[c];
            g.nu[3 * e + c] = n[c];
        }
        if (deg[lo] >= kMaxNbr || deg[hi] >= kMaxNbr)
            throw std::runtime_error("geodesic grid: more than 6 edges");
        g.adj_e[kMaxNbr * lo + deg[lo]] = e;
        g.adj_s[kMaxNbr * lo + deg[lo]++] = +1;
        g.adj_e[kMaxNbr * hi + deg[hi]] = e;
        g.adj_s[kMaxNbr * hi + deg[hi]++] = -1;
        ++e;
    }
    return g;
}

}  // namespace rt
