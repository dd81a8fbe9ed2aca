// Host-only part of the radiation-step library: the angular grids, the
// FP64 geometry tables and the descriptor checks (no HIP types, so these
// sources also build with a plain host compiler).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "rt.h"

namespace rt {

constexpr int kMaxNbr = 6;        // polygon edges per direction (5 or 6)

// ---------------------------------------------------------------- host grid
struct Geodesic {
    int nlev = 0;
    int nang = 0;
    int nedge = 0;
    std::vector<double> nhat;     // [nang][3]
    std::vector<double> domega;   // [nang]
    std::vector<int> lo, hi;      // [nedge]
    std::vector<double> len;      // [nedge]
    std::vector<double> mid;      // [nedge][3]
    std::vector<double> nu;       // [nedge][3]  lo -> hi
    std::vector<int> adj_e;       // [nang][6] edge index or -1
    std::vector<int> adj_s;       // [nang][6] +1 if the direction is the edge's lo, -1 if hi
    std::vector<int> ll, rr;      // [nedge] PLM stencil beyond lo / hi (latitude-longitude only)
};

Geodesic build_geodesic(int nlev);
Geodesic build_latlong(int n_zeta, int n_psi);
// MAPR tables (rt_mapr.cpp): per direction the neighbours in angular order
// [nang][6] (padded with the direction itself), their count, the inverse
// 2x2 matrices of the candidate planes [nang][6][4]; per edge the midpoint
// offsets from lo and from hi [nedge][4]
void build_mapr(const Geodesic &g, std::vector<int> &nb, std::vector<double> &inv,
                std::vector<int8_t> &cnt, std::vector<double> &d);

// Derived host tables (FP64), geometry-cell major.
struct HostTables {
    int G = 0;                    // geometry cells
    int F[3] = {0, 0, 0};         // faces per family (geometry layout)
    std::vector<double> q;        // [G][nang]   n^0 n_0 (cell centre)
    std::vector<double> C[3];     // [F_a][nang] dA n^a n_0 (face centre)
    std::vector<int8_t> sgn[3];   // [F_a][nang] sign of n^a at the face
    std::vector<uint8_t> mask;    // [G][nang]   |n_0| < n0_crit
    std::vector<double> vw;       // [G][nedge][2] (v, w)
    std::vector<double> n0u;      // [G]         n^0
    std::vector<double> E0;       // [G][4][4]   g_{a mu} e^mu_{b^}
    std::vector<double> gas_map;  // [G][4][4]   T^{0^ b^} = sum_mu gas_map[b][mu] T^0_mu
    std::vector<double> vol;      // [G]
    bool has_edges = false;
    int masked_count = 0;
};

int build_tables(const rt_grid_desc &d, const Geodesic &ang, HostTables &t,
                 std::string &err);

// Descriptor checks of rt_init_grid: RT_OK, or an error code with the
// reason in err.
int check_desc(const rt_grid_desc *d, std::string &err);

}  // namespace rt
