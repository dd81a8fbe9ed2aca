// Internal declarations of the radiation-step library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rt.h"
#include "rt_host.h"

namespace rt {

constexpr int kWave = 64;         // CDNA wavefront
constexpr int kMaxChunks = 8;     // directions per lane: nang <= 512

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
    int own_stride;               // LDS entries of the cell's row
    int col_lds;                  // LDS entries per column (row twice + FP32 edge weights)
    int split;                    // waves per column (1, or 2: FP32 with six chunks)
    size_t tab_bytes;             // LDS bytes of the direction tables (before the waves' parts)
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
// raise a kernel's dynamic-LDS limit on the current device to `bytes` (once
// per device and kernel, thread-safe); a no-op within the default 64 KiB
int ensure_dynamic_lds(const void *kernel, size_t bytes);
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
bool column_config(rt_grid *g, int seglen_hint);
int launch_column(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                  const double *rho, const double *u, const double *ka, const double *ks,
                  double dt, double *dT0, void *Istar, const Partials &P);
// the two-stage integrator on the column path (DC angular fluxes, no tau
// flux or velocity substitute), both stages' finalisers included
int launch_column_rk2(rt_grid *g, hipStream_t s, const void *Iin, void *Iout, double *T,
                      const double *rho, const double *u, const double *ka, const double *ks,
                      double dt, double *dT0, double *lum, const Partials &P);
// k_gas.hip
int launch_gas_update(rt_grid *g, hipStream_t s, const double *dT0, const double *Tpre,
                      double *rho, double *u, double *T, int32_t *status);
}  // namespace rt
