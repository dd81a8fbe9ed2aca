/*
 * rt.h -- C ABI of the MI355X finite-solid-angle GR radiation step.
 *
 * The library advances the gray, discrete-angle intensity of White et al.
 * (2023), "An Extension of the Athena++ Code Framework for Radiation-MHD in
 * General Relativity Using a Finite-Solid-Angle Discretization": the
 * conserved variable Q = n^0 n_0 I on a geodesic (or latitude-longitude)
 * angular grid (Sec. 2.2, gray integral form, Sec. 2.6), moved by upwind
 * spatial fluxes (Sec. 2.3-2.4) and angular fluxes between neighbouring
 * solid angles (DC, MAPR or PLM face values), then coupled implicitly to a
 * gamma-law gas through the fluid-frame quartic (Sec. 2.5); optionally with
 * the two-stage integrator, the optical-depth-aware flux and the
 * radiation-dominated velocity substitute.  rt_step_adjoint reverses the
 * one-stage step; rt_gas_update hands the coupling's four-momentum to the
 * gas.
 *
 * Conventions
 *   - Every call returns int: RT_OK (0) or a negative RT_E* code.  The
 *     message of the last failure on the calling thread is rt_last_error().
 *     No C++ exception or abort crosses the ABI.
 *   - Argument checks run synchronously before any launch; an invalid call
 *     launches nothing and changes nothing.
 *   - Device pointers ("dev") live on the grid's device; host pointers
 *     ("host") are read before the call returns.  Kernels run asynchronously
 *     on the caller's HIP stream (hipStream_t passed as void*; NULL = the
 *     default stream); the caller keeps its buffers alive until that stream
 *     has finished with them.  A launch failure returns RT_EDEVICE.
 *   - Only rt_init_grid allocates device memory; rt_free releases it.  The
 *     library keeps no pointer to caller memory after a call returns.
 *   - Cells are indexed (k, j, i) with axis 0 (i) fastest.  Per-cell arrays
 *     are [n2][n1][n0] (vectors: [..][3], [..][4], ...).  Intensities are
 *     [n2][n1][n0][nang], angle fastest, in the grid's precision (float for
 *     RT_F32, double for RT_F64), without ghost cells: boundary values are
 *     produced inside the kernels from the boundary conditions.
 *   - All thermodynamic and coupling quantities (T, rho, u, kappa, dT0,
 *     luminosity) are double in both precisions.
 *   - Units: c = G = 1; a_rad and k_B/(mu m_p) are descriptor fields.
 */
#ifndef PAPER_2302_04283_RT_H
#define PAPER_2302_04283_RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_grid rt_grid; /* opaque: device tables and scratch */

enum { RT_OK = 0, RT_EINVAL = -1, RT_ENOMEM = -2, RT_EDEVICE = -3, RT_EGEOM = -4 };
enum { RT_F64 = 0, RT_F32 = 1 };             /* intensity path; the solve is always FP64 */
enum { RT_RECON_DC = 0, RT_RECON_PLM = 1 };  /* Sec. 2.3 spatial reconstruction          */
enum { RT_BC_PERIODIC = 0, RT_BC_OUTFLOW_VACUUM = 1 };

/*
 * Problem statement, all host float64, read only during rt_init_grid.
 *
 * Geometry follows Sec. 2.1: the metric g_{ab} in coordinates and a
 * stationary tetrad e^a_{b^} whose time leg is the normal observer,
 * e^a_{0^} = -alpha g^{0a}.  Spatial derivatives of both (d_0 = 0 for a
 * stationary spacetime and tetrad) define the Ricci rotation coefficients
 * (Sec. 2.2) from which the library forms the angular fluxes.
 *
 * Geometry arrays are stored with extent 1 along an axis they do not depend
 * on: geo_extent[a] is 1 or n[a].  A geometry cell index is
 * (gk*g1 + gj)*g0 + gi with g = geo_extent.  Face family a (faces normal to
 * axis a) has extents F[a][b] = g[b] for b != a and, along a,
 * n[a]+1 if g[a] > 1 else 1.
 *
 *   vol[g]         cell volume   int sqrt(-g) dx^1 dx^2 dx^3        (Sec. 2.2)
 *   area[a][f]     face area     int sqrt(-g) dx^b dx^c               (Sec. 2.2)
 *   gcov_c[g][4][4]      g_{mu nu} at the cell centre
 *   dgcov_c[g][3][4][4]  d g_{mu nu} / d x^c, c = 1..3
 *   tet_c[g][4][4]       e^mu_{b^}  (row mu = coordinate index, column b^)
 *   dtet_c[g][3][4][4]   d e^mu_{b^} / d x^c
 *   gcov_f[a][f][4][4], tet_f[a][f][4][4]  the same at face centres
 *   x_faces[a][n[a]+1]   face coordinates (for the time-step rule only)
 *
 * beam_mask (optional, [n2][n1][n0], nonzero = beam cell): after each
 * step the intensity of direction beam_angle in those cells is set to
 * beam_I (a fixed-intensity source).
 *
 * integrator: 1 = one forward-Euler transport stage plus the implicit
 * coupling per step; 2 = the two-stage (Heun) integrator of the paper's
 * multi-stage scheme (Sec. 2 task list; second order in time, Sec. 3
 * diffusion): stage 1 is the one-stage step, stage 2 forms
 * ((U0 + U1) + dt L(U1))/2 and the gas temperature (T0 + T1)/2 and applies the
 * coupling over dt/2; the T^0_alpha bookkeeping, the masked-energy ledger and
 * the luminosity then carry (stage 1)/2 + stage 2.  rt_init_grid allocates
 * one extra state and one cell array for it.
 * tau_coeff: constant of the optical-depth-aware flux (Sec. 2, flux
 * calculation): per face tau = tau_coeff alpha_E dt / u^0^ from the averages
 * of the two adjacent cells, f = -expm1(-tau^2), g_L/R = -f (1 + 1/n0bar_L/R)
 * from each cell's own fluid, g = (g_L + g_R)/2, and the upwind value times
 * 1 + (g - g_up).  0 = free streaming.
 * rad_velocity: radiation-dominated velocity substitute (Sec. 2.5).  In a
 * cell whose fluid-frame radiation energy E (at the gas velocity u) exceeds
 * rho + u_gas, the coupling runs at the velocity u'^a = (1 - f^a) u^a +
 * f^a u_rad^a instead of u: v_rad = R^{0a}/R^{00} (tetrad frame), the force
 * G^a = -(alpha_a a_rad T^4 + alpha_s E) u^a - alpha_E u_b R^{ab},
 * f^a = G^a dt / (n^0 (T_rad^{0a} - T_gas^{0a})) clamped to [0, 1] with
 * T^{0a} = (rho + u_gas + p) u^0 u^a at each velocity and n^0 = 1/lapse
 * (the tetrad-frame time of a coordinate step dt is dt/n^0, so f^a is the
 * share of the momentum gap one step of the force closes; the printed
 * divisor u^a is read as this factor).  Cells with R^{00} <= 0 or
 * |v_rad| >= 1 keep u.  The velocity field itself is not changed by rt_step
 * (see rt_gas_update).
 * n_zeta, n_psi: with n_zeta > 0 the angular grid is the latitude-longitude
 * grid of Sec. 2.6 (nlev is ignored): n_zeta + 1 circles of latitude equally
 * spaced in cos(zeta) (zeta from the tetrad x^3 axis), n_psi + 1 meridians
 * equally spaced in psi (from the x^1 axis), direction n = l n_psi + m at the
 * middle of its cos(zeta) and psi ranges; n_zeta >= 2, n_psi even >= 2,
 * n_zeta n_psi <= 512.
 * ang_recon = 1 (latitude-longitude only): angular fluxes take van Leer PLM
 * face values along the edge's coordinate line (Sec. 2.3), across a pole from
 * the cell of the same row at psi + pi; rt_step_adjoint is then unavailable.
 * ang_recon = 2 (geodesic only): minimum-angle plane reconstruction (MAPR,
 * Sec. 2.6): per direction, in the plane tangent at its centre, the candidate
 * planes through the cell and each pair of consecutive neighbours; the one of
 * smallest gradient gives the face value at each edge midpoint (first of equal
 * minima in angular order); rt_step_adjoint is then unavailable.
 * With integrator 2 or tau_coeff > 0 the step runs the general kernel, and
 * rt_step_adjoint / the I_star output are not available (RT_EINVAL).  With
 * rad_velocity the step runs the general kernel and rt_step_adjoint is not
 * available (RT_EINVAL).
 */
typedef struct {
    int32_t n[3];
    int32_t geo_extent[3];
    int32_t nlev;              /* geodesic level N >= 1: nang = 10 N^2 + 2 (Sec. 2.6) */
    int32_t precision;         /* RT_F32 or RT_F64 */
    int32_t recon;             /* RT_RECON_DC or RT_RECON_PLM */
    int32_t bc[3][2];          /* per axis, (lower, upper) */
    int32_t lum_axis, lum_side;/* face whose outgoing energy flux is the luminosity */
    double n0_crit;            /* |n_0| below which I is zeroed (Sec. 2.4), paper ~0.1 */
    double a_rad;              /* radiation constant */
    double gamma_gas;          /* adiabatic index */
    double kb_mu_mp;           /* k_B / (mu m_p); c_v = kb_mu_mp / (gamma - 1) */
    const double *x_faces[3];
    const double *vol;
    const double *area[3];
    const double *gcov_c, *dgcov_c, *tet_c, *dtet_c;
    const double *gcov_f[3], *tet_f[3];
    const uint8_t *beam_mask;
    double beam_I;
    int32_t beam_angle;
    int32_t integrator;        /* 1 or 2 (0 is taken as 1) */
    double tau_coeff;          /* >= 0; 0 = free streaming */
    int32_t rad_velocity;      /* 1: radiation-dominated velocity substitute in the coupling */
    int32_t n_zeta, n_psi;     /* n_zeta > 0: latitude-longitude grid instead of the geodesic one */
    int32_t ang_recon;         /* angular reconstruction: 0 = DC, 1 = PLM (latitude-longitude),
                                  2 = MAPR (geodesic) */
    int32_t kernel;            /* 0 = the fastest step kernel the problem allows; 1 = always
                                  the general kernel (a reference for the faster ones); 2 = the
                                  column kernel wherever the problem allows it */
    int32_t seglen;            /* cells per workgroup segment along axis 2 of the marching
                                  kernels; 0 = chosen from the grid size */
} rt_grid_desc;

/*
 * Build the angular grid and the geometry tables on `device` (host FP64),
 * upload them, and allocate the step's scratch.  Fails with RT_EGEOM if the
 * tetrad is not orthonormal (|g e e - eta| > 1e-10) or its time leg is not
 * the normal observer; RT_EINVAL on malformed sizes; RT_ENOMEM if device
 * memory runs out.  *out is NULL on failure.
 */
int rt_init_grid(const rt_grid_desc *desc, int device, rt_grid **out);

/*
 * Host-only: the geodesic directions of level nlev in canonical order (the
 * same table rt_angles returns for a grid of that level), nhat[nang][3] and
 * domega[nang], nang = 10 nlev^2 + 2.  Lets a caller choose directions
 * (e.g. a beam's) before building a grid.
 */
int rt_geodesic_angles(int32_t nlev, double *nhat, double *domega);

/*
 * Host-only: the directions of the n_zeta x n_psi latitude-longitude grid in
 * its order (n = l n_psi + m), nhat[nang][3] and domega[nang],
 * nang = n_zeta n_psi.
 */
int rt_latlong_angles(int32_t n_zeta, int32_t n_psi, double *nhat, double *domega);

/*
 * Number of directions and of angular-grid edges, and which step kernel the
 * grid uses: 1 = the tiled kernel for spatially uniform geometry, 2 = the
 * column kernel for geometry independent of axis 2 (one-stage step, DC
 * angular fluxes), 0 = the general kernel.  Any output may be NULL.
 */
int rt_grid_info(const rt_grid *g, int32_t *nang, int32_t *nedge, int32_t *fast_path);

/*
 * The angular grid in its canonical order (rings of equal polar angle from
 * the +x^3 pole, each ring by azimuth from -0.01 rad): unit directions
 * nhat[nang][3] and solid angles domega[nang] (host, caller-allocated).
 */
int rt_angles(const rt_grid *g, double *nhat, double *domega);

/*
 * Largest stable step for Courant number cfl:
 *   dt = cfl * min_{cells, dirs} min( min_a dx^a n^0/|n^a|,
 *                                     dOmega n^0 / sum_{outflow edges} |v| ).
 * (The paper gives no rule; this per-direction Courant limit is ours.)
 */
int rt_max_dt(const rt_grid *g, double cfl, double *dt);

/*
 * One step (Sec. 2 task order: fluxes -> flux divergence -> primitives ->
 * implicit coupling), out of place:
 *   I_in  (dev, const)  intensities at the start of the step
 *   I_out (dev)         intensities after the step (must not alias I_in)
 *   T     (dev, in/out) gas temperature [cells]
 *   rho, kappa_a, kappa_s (dev) [cells]; u_tet (dev) tetrad-frame u^{a^} [cells][3]
 *   dt    coordinate time step (> 0)
 *   dT0   (dev, optional) [cells][4], += the change of T^0_alpha that
 *         balances the radiation four-momentum exchanged by the coupling
 *         (Sec. 2.5, last paragraph); NULL to skip
 *   lum   (dev, optional) one double, += dt * (energy per unit time leaving
 *         through the luminosity face); NULL to skip
 *   I_star (dev, optional) [n2][n1][n0][nang], grid precision: receives the
 *         intensities after transport and before the coupling (I*, zero for
 *         masked directions), which rt_step_adjoint can take instead of
 *         recomputing the transport; must not alias I_in or I_out; NULL to skip
 * Directions with |n_0| < n0_crit leave the step with zero intensity.
 */
int rt_step(rt_grid *g, void *stream, const void *I_in, void *I_out, double *T,
            const double *rho, const double *u_tet, const double *kappa_a,
            const double *kappa_s, double dt, double *dT0, double *lum, void *I_star);

/*
 * rt_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, the same kernels and bit-identical results, but the
 * per-block partial sums that rt_step leaves in the grid's buffer for its
 * final fixed-order reduction (luminosity, masked energy, quartic failures)
 * go to a static device array of the library instead: 16 MiB per GPU,
 * present on every GPU the library runs on until the process ends.  The
 * call allocates nothing and frees nothing.
 *   Limit: 2 doubles + 1 int per workgroup of the step's largest launch;
 *   a grid whose step needs more (more than about 13 million cells on the
 *   general kernel) is rejected with RT_EINVAL before any launch.
 *   All calls on one GPU share that array (every block rewrites its own
 *   slots before they are read, so nothing carries over from a previous
 *   call); calls that overlap on one GPU, on any streams or grids, race.
 *   RT_EDEVICE if the array's device address could not be looked up when
 *   the grid was built.
 */
int rt_step_noalloc(rt_grid *g, void *stream, const void *I_in, void *I_out, double *T,
                    const double *rho, const double *u_tet, const double *kappa_a,
                    const double *kappa_s, double dt, double *dT0, double *lum, void *I_star);

/*
 * Adjoint of rt_step for the functional J = sum over steps of
 * w_s * dt * l(I_s), l the luminosity of rt_step: the step of Sec. 2.2-2.5
 * (transport of Sec. 2.3-2.4, coupling of Sec. 2.5) differentiated in
 * reverse order, for gradients of the outgoing luminosity with respect to
 * the opacities, the gas temperature and the intensities.  Given the state at the
 * start of step s (I_n, T_n, the same fluid, opacities and dt) and
 * lamI_np1 = dJ/dI_{s+1}, lamT_np1 = dJ/dT_{s+1}, it writes
 * lamI_n = dJ/dI_s and lamT_n = dJ/dT_s and adds this step's share of
 * dJ/dkappa_a and dJ/dkappa_s.  lum_weight is w_s (1 for J = sum dt l).
 * The quartic is reversed with the implicit-function theorem; the PLM
 * limiter with its Jacobian on the branch the forward step took.
 *   I_n, lamI_np1, lamI_n, work (dev) [n2][n1][n0][nang], grid precision;
 *     lamI_n may alias lamI_np1 (read completely before lamI_n is written);
 *     work is caller-owned scratch of the same size, not aliasing the others
 *   T_n, lamT_np1, lamT_n (dev) [cells]; lamT_n may alias lamT_np1
 *   grad_kappa_a, grad_kappa_s (dev) [cells], accumulated (+=), or NULL
 *   I_star (dev, optional, const) I* of this step as written by rt_step's
 *     I_star output for the same inputs; when given, the transport is not
 *     recomputed (the caller guarantees it matches I_n); NULL to recompute
 */
int rt_step_adjoint(rt_grid *g, void *stream, const void *I_n, const double *T_n,
                    const double *rho, const double *u_tet, const double *kappa_a,
                    const double *kappa_s, double dt, double lum_weight, const void *lamI_np1,
                    const double *lamT_np1, void *lamI_n, double *lamT_n, void *work,
                    double *grad_kappa_a, double *grad_kappa_s, const void *I_star);

/*
 * Radiation moments per cell (Sec. 2.5):
 *   R_tet  [cells][10]  R^{a^ b^} = sum_n I n^{a^} n^{b^} dOmega, pairs
 *                       00 01 02 03 11 12 13 22 23 33 (tetrad frame)
 *   R0_cov [cells][4]   R^0_alpha = sum_n n^0 n_alpha I dOmega (coordinate)
 *   E_fluid [cells]     fluid-frame energy density sum_n I (n^0bar)^2 dOmega
 * Any output may be NULL.  All dev.
 */
int rt_moments(rt_grid *g, void *stream, const void *I, const double *u_tet,
               double *R_tet, double *R0_cov, double *E_fluid);

/*
 * Hands the four-momentum the coupling took from the radiation to a
 * gamma-law gas (Sec. 2.5, last paragraph: the change of R^0_alpha is
 * subtracted from the gas's T^0_alpha).  Per cell, T^0_alpha of the gas
 * state (rho, u_tet, T_pre) plus dT0 is inverted for the new primitive state
 * with rho u^0 held (the coupling does not change the conserved density):
 * in the normal-observer tetrad frame D = rho u^0^, E = T^{0^0^},
 * S = T^{0^a^}; p solves (D/gamma + Gamma p/(Gamma-1)) gamma^2 - p = E with
 * v = |S|/(E + p); then rho = D/gamma, u^a^ = gamma S/(E + p), T = p/(rho kb).
 *   dT0   (dev, const) [cells][4] the change of T^0_alpha of ONE rt_step
 *         (the caller zeroes it before that step)
 *   T_pre (dev, const) [cells] gas temperature at the start of that step
 *   rho, u_tet, T (dev, in/out) [cells], [cells][3], [cells]; T may alias T_pre
 *   status (dev, optional) [cells] int32: 0 = updated, 1 = no physical state
 *         (energy below momentum or rest mass + kinetic energy; the cell's
 *         rho, u_tet, T are left unchanged)
 * Gas parameters (gamma_gas, kb_mu_mp) are the grid's.
 */
int rt_gas_update(rt_grid *g, void *stream, const double *dT0, const double *T_pre,
                  double *rho, double *u_tet, double *T, int32_t *status);

/*
 * Running totals since rt_init_grid (synchronises the grid's device):
 * number of cells whose quartic of Sec. 2.5 had no positive root (T set to
 * 1e-12), and the energy removed by the |n_0| mask of Sec. 2.4 (directions
 * too close to the horizon, whose primitive intensity is set to zero).
 */
int rt_stats(rt_grid *g, int64_t *no_root_events, double *masked_energy);

/* Release every device table and scratch buffer of g (NULL is a no-op). */
void rt_free(rt_grid *g);

/* Message of the last failure on this thread ("" if none). */
const char *rt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
