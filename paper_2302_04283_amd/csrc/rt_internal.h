// Internal declarations of the radiation-step library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rt.h"

namespace rt {

constexpr int kMaxNbr = 6;        // polygon edges per direction (5 or 6)
constexpr int kWave = 64;         // CDNA wavefront
constexpr int kMaxChunks = 8;     // directions per lane: nang <= 512

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

// ---------------------------------------------------------------- device view
struct DevGrid {
    int n0, n1, n2, nang, nedge;
    int g0, g1, g2;
    int fe[3][3];                 // face-family extents [family][axis]
    int bc[3][2];
    int recon;
    int lum_axis, lum_side;
    double a_rad, cv;
    double kb, gamma;             // k_B / mu m_p, adiabatic index
    double tau_coeff;             // optical-depth-aware flux constant (0 = off)
    int rad_velocity;             // radiation-dominated velocity substitute
    // angle tables
    const double *nhat;           // [nang][3]
    const double *domega;         // [nang]
    const int *adj_e;             // [nang][6]
    const int *adj_s;             // [nang][6]
    const int *edge_lo, *edge_hi; // [nedge]
    const int *edge_ll, *edge_rr; // [nedge] angular PLM stencil, or nullptr
    int ang_recon;                // 0 = DC, 1 = PLM (latitude-longitude), 2 = MAPR (geodesic)
    const int *mapr_nb;           // [nang][6]
    const int8_t *mapr_cnt;       // [nang]
    const void *mapr_inv;         // [nang][6][4] intensity precision
    const void *mapr_d;           // [nedge][4]   intensity precision
    // geometry tables in the intensity precision
    const void *q;                // [G][nang]
    const void *C[3];             // [F_a][nang]
    const void *vw;               // [G][nedge][2]
    const void *invV;             // [G]
    const int8_t *sgn[3];         // [F_a][nang]
    const uint8_t *mask;          // [G][nang]
    const double *n0u;            // [G]
    const double *E0;             // [G][16]
    const double *gas_map;        // [G][16]
    const double *volD;           // [G]
    int has_edges;
    const uint8_t *beam;          // [cells] or nullptr
    int beam_angle;
    double beam_I;
};

// Where a step's kernels leave their per-block partial sums (luminosity,
// masked energy, quartic failures) for the finaliser: the grid's own buffer,
// or the device-static scratch of rt_step_noalloc.
struct Partials {
    double *sums;                 // [blocks][2]
    int *noroot;                  // [blocks]
};

// Fast path for spatially uniform geometry (k_march.hip).
struct MarchInfo {
    int enabled;
    int sw, nc;                   // lane-group width, directions per lane
    int ntx, nseg, seglen, nwork, grid;
    int pstride;                  // LDS stride of a plane cell
    int any_mask;                 // some direction is masked
    size_t lds;                   // dynamic LDS bytes
    const void *q, *iq, *cx, *cy, *cz;   // per-direction tables (intensity precision)
    const uint8_t *bits;          // per-direction sign/mask flags
    double vol;
};

// Column march for geometry independent of axis 2 (k_column.hip).
struct ColumnInfo {
    int enabled;
    int seglen, nseg, grid;
    long long nwork;              // column segments (one wavefront each)
    int own_stride;               // LDS entries of a wave's own row
    int wave_lds;                 // LDS entries per wave (own row + FP32 edge weights)
};

}  // namespace rt

struct rt_grid {
    int device = 0;
    int precision = RT_F64;
    rt::Geodesic ang;
    rt::DevGrid dg{};
    rt::MarchInfo march{};
    rt::ColumnInfo column{};
    std::vector<double> dx[3];    // coordinate widths (for rt_max_dt)
    std::vector<double> host_n0u; // [G]
    std::vector<double> host_na;  // [G][nang][3] n^a at centres (for rt_max_dt)
    std::vector<double> host_vw;  // [G][nedge][2]
    std::vector<void *> allocs;   // every device allocation
    // scratch
    void *scratch = nullptr;      // this device's static scratch (rt_step_noalloc)
    size_t scratch_bytes = 0;
    double *partials = nullptr;   // [max_blocks][2]
    int *noroot_partial = nullptr;// [max_blocks]
    double *ledger = nullptr;     // [1] masked energy
    long long *noroot = nullptr;  // [1]
    int max_blocks = 0;
    int integrator = 1;           // 1 or 2 stages per step
    void *stage_I = nullptr;      // two-stage integrator: stage-1 intensities
    double *stage_T = nullptr;    //                       stage-1 temperature
};

// kernel launchers (k_step.hip)
namespace rt {
int launch_step(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                const double *rho, const double *u, const double *ka, const double *ks,
                double dt, double *dT0, double *lum, void *Istar, const Partials &P);
int launch_moments(rt_grid *g, hipStream_t s, const void *I, const double *u,
                   double *R, double *R0, double *E);
int step_blocks(const rt_grid *g);
// blocks whose partial sums one step writes (the largest launch of the step)
int step_partial_blocks(const rt_grid *g);
// device address of this device's static scratch (the calling thread's
// current device); looked up once per device
int scratch_address(void **ptr, size_t *bytes);
bool march_config(int precision, int nang, int &sw, int &nc);
size_t march_lds_bytes(int precision, int nang, int np);
int march_pstride(int precision, int nang);
int launch_march(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                 const double *rho, const double *u, const double *ka, const double *ks,
                 double dt, double *dT0, void *Istar, const Partials &P);
int launch_finalize(rt_grid *g, hipStream_t s, int nblocks, double dt, double *lum,
                    const Partials &P);
bool march_rk2_config(int sw, int nc);
int launch_march_rk2(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                     const double *rho, const double *u, const double *ka, const double *ks,
                     double dt, double *dT0, double *lum, const Partials &P);
int launch_adjoint(rt_grid *g, hipStream_t s, const void *Iin, const double *Tin,
                   const double *rho, const double *u, const double *ka, const double *ks,
                   double dt, double lum_weight, const void *lamI1, const double *lamT1,
                   void *lamI0, double *lamT0, void *work, double *gka, double *gks,
                   const void *Istar);
int launch_adj_march(rt_grid *g, hipStream_t s, const void *Iin, const void *psi, double dt,
                     double lum_weight, void *lamI0);
// k_adj_column.hip: the transport adjoint with the column layout (used where
// the forward step uses k_column)
int launch_adj_column(rt_grid *g, hipStream_t s, const void *Iin, const void *psi, double dt,
                      double lum_weight, void *lamI0);
// k_column.hip
bool column_config(rt_grid *g, int seglen_hint, bool force);
int launch_column(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                  const double *rho, const double *u, const double *ka, const double *ks,
                  double dt, double *dT0, void *Istar, const Partials &P);
// k_gas.hip
int launch_gas_update(rt_grid *g, hipStream_t s, const double *dT0, const double *Tpre,
                      double *rho, double *u, double *T, int32_t *status);
}  // namespace rt
