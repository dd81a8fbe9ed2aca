"""Seeded synthetic problem statements for the radiation step.

This module is the only code shared by the HIP path and the CPU oracle.  It
builds what the paper calls the *statement of the problem* and nothing of the
scheme itself:

* a counter-based random generator (splitmix64, Steele, Lea & Flood 2014) so
  that any field value is a pure function of (seed, field id, global index)
  and any sub-box can be regenerated bit-identically;
* spatial grids (face coordinates, cell centres);
* the spacetime metric g_{ab} in coordinates and its spatial derivatives,
  the normal-observer tetrad e^a_{b^} (time leg -alpha g^{0a}, Sec. 2.1) and
  its derivatives, at cell centres and face centres;
* cell volumes and face areas, the sqrt(-g)-weighted measures of Sec. 2.2;
* fluid state (rho, tetrad-frame u^{a^}, T), opacities and initial
  intensities.

It holds no step of the method: no angular grid, no Ricci rotation
coefficients, no fluxes, no coupling.  Derivatives of the metric and tetrad
are obtained by complex-step differentiation of the closed forms, which is
exact to round-off for these analytic expressions.

Layout conventions (shared by both sides, documented in the C header):
per-cell arrays are [n2][n1][n0] (axis 0 fastest); intensities are
[n2][n1][n0][nang] (angle fastest).  Geometry arrays are stored with extent 1
along any axis they do not depend on (``geo_extent``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# ----------------------------------------------------------------------------
# counter-based generator
# ----------------------------------------------------------------------------
_MASK = np.uint64(0xFFFFFFFFFFFFFFFF)
SEED_BASE = 230204283

# field identifiers (bits 56..63 of the counter)
F_T = 1
F_INOISE = 2
F_RHO = 3          # normal pair 3,4
F_TAU_A = 5        # normal pair 5,6
F_TAU_S = 7        # normal pair 7,8
F_VDIR = 9         # three normal pairs 9..14
F_VMAG = 15
F_VPERT = 16       # three uniforms 16,17,18


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 output function applied to counter values ``x`` (uint64)."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _MASK
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _MASK
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _MASK
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, fid: int, idx: np.ndarray) -> np.ndarray:
    """U[0,1) doubles: top 53 bits of splitmix64(seed ^ fid<<56 ^ idx)."""
    idx = np.asarray(idx, dtype=np.uint64)
    key = np.uint64(seed) ^ (np.uint64(fid) << np.uint64(56))
    r = splitmix64(idx ^ key)
    return (r >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, fid: int, idx: np.ndarray) -> np.ndarray:
    """Standard normals by Box-Muller over the field pair (fid, fid+1)."""
    u1 = uniform(seed, fid, idx)
    u2 = uniform(seed, fid + 1, idx)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


# ----------------------------------------------------------------------------
# spacetimes: metric and normal-observer tetrad, complex-analytic in (x1, x2)
# ----------------------------------------------------------------------------

def _metric_minkowski_cart(x1, x2, x3):
    shp = np.broadcast(x1, x2, x3).shape
    g = np.zeros(shp + (4, 4), dtype=np.result_type(x1, x2, x3, np.float64))
    g[..., 0, 0] = -1.0
    g[..., 1, 1] = g[..., 2, 2] = g[..., 3, 3] = 1.0
    return g


def _metric_kerr_schild_sph(M, a):
    """Spherical Kerr-Schild metric (t, r, theta, phi), mass M, spin a."""
    def g_of(r, th, ph):
        r, th, ph = np.broadcast_arrays(r, th, ph)
        s = np.sin(th)
        c = np.cos(th)
        sig = r * r + a * a * c * c
        f = 2.0 * M * r / sig
        g = np.zeros(r.shape + (4, 4), dtype=np.result_type(r, th, np.float64))
        g[..., 0, 0] = -(1.0 - f)
        g[..., 0, 1] = g[..., 1, 0] = f
        g[..., 0, 3] = g[..., 3, 0] = -f * a * s * s
        g[..., 1, 1] = 1.0 + f
        g[..., 1, 3] = g[..., 3, 1] = -a * (1.0 + f) * s * s
        g[..., 2, 2] = sig
        g[..., 3, 3] = (r * r + a * a + f * a * a * s * s) * s * s
        return g
    return g_of


def normal_tetrad(g: np.ndarray) -> np.ndarray:
    """Tetrad e[..., mu, b^] with time leg -alpha g^{0 mu} (normal observer)
    and spatial legs by Gram-Schmidt of (d_1, d_2, d_3) under gamma_ab.
    Uses the complex-analytic bilinear form (no conjugation) so it can be
    complex-step differentiated."""
    ginv = np.linalg.inv(g)
    alpha = 1.0 / np.sqrt(-ginv[..., 0, 0])
    e = np.zeros_like(g)
    e[..., :, 0] = -alpha[..., None] * ginv[..., 0, :]
    gam = g[..., 1:, 1:]

    def dot(v, w):
        return np.einsum("...i,...ij,...j->...", v, gam, w)

    basis = []
    for k in range(3):
        v = np.zeros(g.shape[:-2] + (3,), dtype=g.dtype)
        v[..., k] = 1.0
        for b in basis:
            v = v - dot(v, b)[..., None] * b
        v = v / np.sqrt(dot(v, v))[..., None]
        basis.append(v)
    for k in range(3):
        e[..., 1:, k + 1] = basis[k]
    return e


def _with_derivs(fn, x1, x2, x3, dep, h=1e-20):
    """Value and spatial derivatives [..., 3, ...] of fn by complex step.
    ``dep`` lists the coordinate axes fn depends on (others: zero)."""
    val = np.real(fn(x1 + 0j, x2 + 0j, x3 + 0j))
    d = np.zeros(val.shape[:-2] + (3,) + val.shape[-2:])
    xs = [x1, x2, x3]
    for ax in dep:
        xx = [np.asarray(v, dtype=np.complex128) for v in xs]
        xx[ax] = xx[ax] + 1j * h
        d[..., ax, :, :] = np.imag(fn(*xx)) / h
    return val, d


# ----------------------------------------------------------------------------
# problem container
# ----------------------------------------------------------------------------
BC_PERIODIC = 0
BC_OUTFLOW_VACUUM = 1
RECON_DC = 0
RECON_PLM = 1


@dataclass
class Problem:
    """Everything a radiation step needs, as host float64 numpy arrays."""
    name: str
    n: tuple                      # active cells (n0, n1, n2), axis 0 fastest
    geo_extent: tuple             # 1 or n[a] per axis
    nlev: int
    recon: int
    bc: tuple                     # ((lo, hi) for axis 0, 1, 2)
    x_faces: list                 # 3 arrays of n[a]+1 face coordinates
    # geometry at cell centres, arrays [g2][g1][g0][...]
    gcov_c: np.ndarray            # [..,4,4]
    dgcov_c: np.ndarray           # [..,3,4,4]  d_{x^c} g_{ab}, c = 1..3
    tet_c: np.ndarray             # [..,4,4]    e^mu_{b^}
    dtet_c: np.ndarray            # [..,3,4,4]  d_{x^c} e^mu_{b^}
    vol: np.ndarray               # [g2][g1][g0]
    # geometry at face centres of family a
    gcov_f: list                  # 3 x [..,4,4]
    tet_f: list                   # 3 x [..,4,4]
    area: list                    # 3 x [f2][f1][f0]
    # fluid and opacities, per active cell [n2][n1][n0]
    rho: np.ndarray
    u_tet: np.ndarray             # [n2][n1][n0][3] tetrad-frame u^{a^}
    T: np.ndarray
    kappa_a: np.ndarray
    kappa_s: np.ndarray
    # physical constants and scheme parameters
    n0_crit: float = 0.1
    a_rad: float = 1.0
    gamma_gas: float = 5.0 / 3.0
    kb_mu_mp: float = 1.0
    lum_axis: int = 0
    lum_side: int = 1
    cfl: float = 0.3
    nsteps: int = 10
    # time integrator: 1 = one forward-Euler stage per step, 2 = two-stage
    # (Heun) integrator; optical-depth-aware flux constant (0 = free streaming)
    integrator: int = 1
    tau_coeff: float = 0.0
    # radiation-dominated velocity substitute in the coupling (0 = off)
    rad_velocity: int = 0
    # angular grid: None = geodesic of level nlev; (n_zeta, n_psi) = the
    # latitude-longitude grid; angular reconstruction 0 = DC, 1 = PLM
    # (latitude-longitude only)
    latlong: Optional[tuple] = None
    ang_recon: int = 0
    # step kernel: 0 = the fastest one the problem allows, 1 = the general
    # kernel, 2 = the column kernel wherever allowed; cells per workgroup
    # segment along axis 2 (0 = automatic)
    kernel: int = 0
    seglen: int = 0
    # optional fixed-intensity beam cells
    beam_mask: Optional[np.ndarray] = None   # [n2][n1][n0] bool
    beam_I: float = 0.0
    # bookkeeping for regeneration
    seed: int = SEED_BASE
    origin: tuple = (0, 0, 0)     # global index of cell (0,0,0) of this box
    global_n: tuple = None        # full-domain cell counts
    extras: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nang(self) -> int:
        if self.latlong is not None:
            return int(self.latlong[0] * self.latlong[1])
        return 10 * self.nlev * self.nlev + 2

    def global_cell_index(self) -> np.ndarray:
        """Global linear index (k*N1 + j)*N0 + i of every active cell."""
        N0, N1, N2 = self.global_n
        i = (self.origin[0] + np.arange(self.n[0])) % N0
        j = (self.origin[1] + np.arange(self.n[1])) % N1
        k = (self.origin[2] + np.arange(self.n[2])) % N2
        return ((k[:, None, None] * N1 + j[None, :, None]) * N0
                + i[None, None, :]).astype(np.uint64)

    def initial_intensity(self, dtype=np.float64, k_range=None) -> np.ndarray:
        """I = a_rad T^4/(4 pi) (1 + 0.1 xi), xi ~ U[0,1) per (cell, angle),
        isotropic in the tetrad frame.  ``k_range`` selects axis-2 slabs."""
        nang = self.nang
        gidx = self.global_cell_index()
        T = self.T
        if k_range is not None:
            gidx = gidx[k_range[0]:k_range[1]]
            T = T[k_range[0]:k_range[1]]
        ang = np.arange(nang, dtype=np.uint64)
        xi = uniform(self.seed, F_INOISE,
                     gidx[..., None] * np.uint64(nang) + ang)
        base = self.a_rad * T ** 4 / (4.0 * math.pi)
        return (base[..., None] * (1.0 + 0.1 * xi)).astype(dtype)

    def initial_intensity_slabs(self, dtype=np.float64, slab=8, workers=8):
        """The same field as ``initial_intensity``, generated as axis-2 slabs
        of ``slab`` planes on a thread pool (numpy releases the GIL) and
        yielded in order as ((k0, k1), array): full-size grids without one
        multi-GB host array."""
        from concurrent.futures import ThreadPoolExecutor
        ranges = [(k, min(self.n[2], k + slab)) for k in range(0, self.n[2], slab)]
        with ThreadPoolExecutor(max(1, workers)) as ex:
            for i in range(0, len(ranges), max(1, workers)):
                part = ranges[i:i + max(1, workers)]
                for kr, arr in zip(part, ex.map(lambda r: self.initial_intensity(dtype, r), part)):
                    yield kr, arr


# ----------------------------------------------------------------------------
# geometry builders
# ----------------------------------------------------------------------------

def _centres(xf):
    return 0.5 * (xf[1:] + xf[:-1])


def _geometry(kind, xf, n, geo_extent, M=0.0, a=0.0):
    """Metric/tetrad (+derivatives) at cell and face centres; volumes/areas."""
    xc = [_centres(v) for v in xf]
    # coordinates of geometry cells (extent 1 -> first cell)
    gc = [xc[ax][: geo_extent[ax]] for ax in range(3)]
    X1, X2, X3 = np.meshgrid(gc[0], gc[1], gc[2], indexing="ij")
    # to [g2][g1][g0]
    X1, X2, X3 = (np.transpose(v, (2, 1, 0)) for v in (X1, X2, X3))
    if kind == "minkowski_cart":
        gfn = _metric_minkowski_cart
        dep = []
    elif kind == "ks_sph":
        gfn = _metric_kerr_schild_sph(M, a)
        dep = [0, 1]
    else:
        raise ValueError(kind)

    def efn(x1, x2, x3):
        return normal_tetrad(gfn(x1, x2, x3))

    g_c, dg_c = _with_derivs(gfn, X1, X2, X3, dep)
    e_c, de_c = _with_derivs(efn, X1, X2, X3, dep)

    g_f, e_f, areas = [], [], []
    for fam in range(3):
        cs = []
        for ax in range(3):
            if ax == fam:
                cs.append(xf[ax] if geo_extent[ax] > 1 else xf[ax][:1])
            else:
                cs.append(gc[ax])
        F1, F2, F3 = np.meshgrid(cs[0], cs[1], cs[2], indexing="ij")
        F1, F2, F3 = (np.transpose(v, (2, 1, 0)) for v in (F1, F2, F3))
        gf = np.real(gfn(F1 + 0j, F2 + 0j, F3 + 0j))
        g_f.append(gf)
        e_f.append(np.real(efn(F1 + 0j, F2 + 0j, F3 + 0j)))

    # volumes and areas: exact integrals of sqrt(-g) over cells / faces
    d = [np.diff(v) for v in xf]
    if kind == "minkowski_cart":
        vol = (d[0][: geo_extent[0]][None, None, :]
               * d[1][: geo_extent[1]][None, :, None]
               * d[2][: geo_extent[2]][:, None, None])
        for fam in range(3):
            o = [ax for ax in range(3) if ax != fam]
            A = np.ones((1, 1, 1))
            for ax in o:
                dd = d[ax][: geo_extent[ax]]
                shp = [1, 1, 1]
                shp[2 - ax] = dd.size
                A = A * dd.reshape(shp)
            ff = xf[fam].size if geo_extent[fam] > 1 else 1
            shp = list(A.shape)
            shp[2 - fam] = ff
            areas.append(np.broadcast_to(A, shp).copy())
    else:
        # sqrt(-g) = (r^2 + a^2 cos^2 th) sin th for Kerr-Schild
        r, th, ph = xf
        rlo, rhi = r[:-1], r[1:]
        tlo, thi = th[:-1], th[1:]
        dphi = np.diff(ph)
        Ir2 = (rhi ** 3 - rlo ** 3) / 3.0            # int r^2 dr
        Ir0 = rhi - rlo                              # int dr
        Is = np.cos(tlo) - np.cos(thi)               # int sin dth
        Ic2s = (np.cos(tlo) ** 3 - np.cos(thi) ** 3) / 3.0  # int cos^2 sin
        g0, g1, g2 = geo_extent
        vol = (dphi[:g2][:, None, None]
               * (Ir2[:g0][None, None, :] * Is[:g1][None, :, None]
                  + a * a * Ir0[:g0][None, None, :] * Ic2s[:g1][None, :, None]))
        # r-faces: [g2][g1][nr+1 or 1]
        rr = r if g0 > 1 else r[:1]
        A0 = dphi[:g2][:, None, None] * (rr[None, None, :] ** 2 * Is[:g1][None, :, None]
                                         + a * a * Ic2s[:g1][None, :, None])
        # theta-faces: [g2][nth+1 or 1][g0]
        tt = th if g1 > 1 else th[:1]
        A1 = dphi[:g2][:, None, None] * np.sin(tt)[None, :, None] * (
            Ir2[:g0][None, None, :] + a * a * np.cos(tt)[None, :, None] ** 2
            * Ir0[:g0][None, None, :])
        # phi-faces: [nph+1 or 1][g1][g0]
        f2 = ph.size if g2 > 1 else 1
        A2 = np.broadcast_to(Ir2[:g0][None, None, :] * Is[:g1][None, :, None]
                             + a * a * Ir0[:g0][None, None, :] * Ic2s[:g1][None, :, None],
                             (f2, g1, g0)).copy()
        areas = [A0, A1, A2]
    return dict(gcov_c=g_c, dgcov_c=dg_c, tet_c=e_c, dtet_c=de_c, vol=vol,
                gcov_f=g_f, tet_f=e_f, area=areas)


def _sub_faces(xf_full, lo, m, periodic, period):
    """Face coordinates of a sub-box [lo, lo+m) with periodic unwrapping."""
    n = xf_full.size - 1
    idx = lo + np.arange(m + 1)
    if periodic:
        wraps = np.floor_divide(idx, n)
        return xf_full[idx % n] + wraps * period
    if lo < 0 or lo + m > n:
        raise ValueError("non-periodic sub-box out of range")
    return xf_full[lo: lo + m + 1].copy()


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def _fluid_minkowski(seed, gidx, kind):
    if kind == "c1":
        T = 0.5 + uniform(seed, F_T, gidx)
        rho = np.ones_like(T)
        u = np.zeros(T.shape + (3,))
        return rho, u, T
    # c2: v uniform in the ball |v| <= 0.5
    dvec = np.stack([normal(seed, F_VDIR + 2 * c, gidx) for c in range(3)], -1)
    dvec = dvec / np.linalg.norm(dvec, axis=-1, keepdims=True)
    vmag = 0.5 * np.cbrt(uniform(seed, F_VMAG, gidx))
    v = dvec * vmag[..., None]
    gam = 1.0 / np.sqrt(1.0 - vmag ** 2)
    u = v * gam[..., None]
    rho = np.exp(normal(seed, F_RHO, gidx))
    T = 0.5 + 1.5 * uniform(seed, F_T, gidx)
    return rho, u, T


def _lognormal_tau(seed, fid, gidx, mu, sig, lo, hi):
    return np.clip(np.exp(mu + sig * normal(seed, fid, gidx)), lo, hi)


def make_problem(cfg: str, scale: Optional[tuple] = None,
                 sub: Optional[tuple] = None, nlev: Optional[int] = None,
                 recon: int = RECON_PLM) -> Problem:
    """Build one of the named workloads.

    cfg:   'c1' .. 'c5': Minkowski 16^3 x 42 (c1) and 128^3 x 162 with a beam
           (c2); Kerr-Schild 128x64x128 x 162 (c3), 64x32x64 x 92 (c4) and
           256x128x256 x 362 with an optically thick torus (c5).
    scale: override of the full-domain cell counts (n0, n1, n2); the recipe
           is otherwise unchanged (used for small parity cases).
    sub:   ((i0, i1, i2), (m0, m1, m2)) sub-box of the full domain; fields are
           regenerated from their global indices, so a sub-box is bit-identical
           to the same cells of the full problem.
    """
    seed = SEED_BASE + int(cfg[1:])
    if cfg in ("c1", "c2"):
        N = {"c1": (16, 16, 16), "c2": (128, 128, 128)}[cfg]
        lev = {"c1": 2, "c2": 4}[cfg]
        steps = {"c1": 10, "c2": 100}[cfg]
        kind = "minkowski_cart"
        bounds = [(0.0, 1.0)] * 3
        bc_full = ((BC_PERIODIC, BC_PERIODIC),) * 3
        periodic = (True, True, True)
        M = a = 0.0
    elif cfg in ("c3", "c4", "c5"):
        N = {"c3": (128, 64, 128), "c4": (64, 32, 64), "c5": (256, 128, 256)}[cfg]
        lev = {"c3": 4, "c4": 3, "c5": 6}[cfg]
        steps = {"c3": 50, "c4": 50, "c5": 20}[cfg]
        kind = "ks_sph"
        bounds = [(1.3, 50.0), (math.pi / 16, 15 * math.pi / 16), (0.0, 2 * math.pi)]
        bc_full = ((BC_OUTFLOW_VACUUM, BC_OUTFLOW_VACUUM),
                   (BC_OUTFLOW_VACUUM, BC_OUTFLOW_VACUUM),
                   (BC_PERIODIC, BC_PERIODIC))
        periodic = (False, False, True)
        M, a = 1.0, 0.9
    else:
        raise ValueError(cfg)
    if scale is not None:
        N = tuple(scale)
    if nlev is not None:
        lev = nlev

    # full-domain face coordinates
    xf_full = []
    for ax in range(3):
        lo, hi = bounds[ax]
        t = np.arange(N[ax] + 1) / N[ax]
        if kind == "ks_sph" and ax == 0:
            xf_full.append(lo * (hi / lo) ** t)
        else:
            xf_full.append(lo + (hi - lo) * t)
        if periodic[ax]:
            xf_full[-1][-1] = hi

    if sub is None:
        origin, n = (0, 0, 0), tuple(N)
        xf = xf_full
        bc = bc_full
    else:
        origin, n = tuple(sub[0]), tuple(sub[1])
        xf = [_sub_faces(xf_full[ax], origin[ax], n[ax], periodic[ax],
                         bounds[ax][1] - bounds[ax][0]) for ax in range(3)]
        # a sub-box is evolved with outflow/vacuum ghosts; only cells outside
        # the halo are compared
        bc = ((BC_OUTFLOW_VACUUM, BC_OUTFLOW_VACUUM),) * 3
        if all(n[ax] == N[ax] and periodic[ax] for ax in range(3)):
            bc = bc_full

    if kind == "minkowski_cart":
        # uniform Cartesian spacing: geometry independent of every axis
        geo_extent = (1, 1, 1)
    else:
        geo_extent = (n[0], n[1], 1)

    geo = _geometry(kind, xf, n, geo_extent, M, a)

    prob_stub = Problem(name=cfg, n=n, geo_extent=geo_extent, nlev=lev, recon=recon,
                        bc=bc, x_faces=xf, rho=None, u_tet=None, T=None,
                        kappa_a=None, kappa_s=None, seed=seed, origin=origin,
                        global_n=tuple(N), nsteps=steps, **geo)
    gidx = prob_stub.global_cell_index()
    xc = [_centres(v) for v in xf]
    if kind == "minkowski_cart":
        if cfg == "c1":
            rho, u, T = _fluid_minkowski(seed, gidx, "c1")
            ka = np.ones_like(T)
            ks = np.zeros_like(T)
        else:
            rho, u, T = _fluid_minkowski(seed, gidx, "c2")
            dx = (bounds[0][1] - bounds[0][0]) / N[0]
            ta = _lognormal_tau(seed, F_TAU_A, gidx, math.log(0.1), 1.5, 1e-3, 10.0)
            ts = _lognormal_tau(seed, F_TAU_S, gidx, math.log(0.1), 1.5, 1e-3, 10.0)
            ka = ta / (rho * dx)
            ks = ts / (rho * dx)
            # beam cells: global i == 0, (y-1/2)^2 + (z-1/2)^2 < 0.1^2
            gi = (origin[0] + np.arange(n[0])) % N[0]
            yy = xc[1][None, :, None]
            zz = xc[2][:, None, None]
            yy = np.mod(yy, 1.0)
            zz = np.mod(zz, 1.0)
            bm = ((gi[None, None, :] == 0)
                  & ((yy - 0.5) ** 2 + (zz - 0.5) ** 2 < 0.01))
            prob_stub.beam_mask = np.broadcast_to(bm, (n[2], n[1], n[0])).copy()
            prob_stub.beam_I = 10.0
    else:
        R = np.broadcast_to(xc[0][None, None, :], (n[2], n[1], n[0]))
        TH = np.broadcast_to(xc[1][None, :, None], (n[2], n[1], n[0]))
        v3 = np.minimum(0.7, R ** -0.5)
        v = np.zeros(R.shape + (3,))
        v[..., 2] = v3
        vm = np.abs(v3)
        for c in range(3):
            xi = 2.0 * uniform(seed, F_VPERT + c, gidx) - 1.0
            v[..., c] += 0.1 * vm * xi
        vn = np.linalg.norm(v, axis=-1)
        cap = np.minimum(1.0, 0.75 / vn)
        v = v * cap[..., None]
        vn = np.linalg.norm(v, axis=-1)
        u = v / np.sqrt(1.0 - vn ** 2)[..., None]
        rho = (1.3 / R) ** 1.5
        T = 1.3 / R
        # minimum proper cell width from the diagonal of gamma at the centre
        g = geo["gcov_c"]
        d = [np.diff(v_) for v_ in xf]
        w0 = np.sqrt(g[..., 1, 1]) * d[0][None, None, : geo_extent[0]]
        w1 = np.sqrt(g[..., 2, 2]) * d[1][None, : geo_extent[1], None]
        w2 = np.sqrt(g[..., 3, 3]) * d[2][: geo_extent[2], None, None]
        dxp = np.broadcast_to(np.minimum(np.minimum(w0, w1), w2), R.shape)
        if cfg == "c5":
            torus = (R * np.sin(TH) - 12.0) ** 2 + (R * np.cos(TH)) ** 2 < 36.0
            rho = np.where(torus, 100.0 * rho, rho)
            ta = np.where(torus,
                          _lognormal_tau(seed, F_TAU_A, gidx, 0.0, 1.5, 1e-3, 100.0),
                          _lognormal_tau(seed, F_TAU_A, gidx, math.log(0.1), 1.5, 1e-3, 10.0))
            ts = np.where(torus,
                          _lognormal_tau(seed, F_TAU_S, gidx, math.log(10.0), 1.5, 1e-3, 100.0),
                          _lognormal_tau(seed, F_TAU_S, gidx, math.log(0.1), 1.5, 1e-3, 10.0))
        else:
            ta = _lognormal_tau(seed, F_TAU_A, gidx, math.log(0.1), 1.5, 1e-3, 10.0)
            ts = _lognormal_tau(seed, F_TAU_S, gidx, math.log(0.1), 1.5, 1e-3, 10.0)
        ka = ta / (rho * dxp)
        ks = ts / (rho * dxp)
    prob_stub.rho = np.ascontiguousarray(rho, dtype=np.float64)
    prob_stub.u_tet = np.ascontiguousarray(u, dtype=np.float64)
    prob_stub.T = np.ascontiguousarray(T, dtype=np.float64)
    prob_stub.kappa_a = np.ascontiguousarray(ka, dtype=np.float64)
    prob_stub.kappa_s = np.ascontiguousarray(ks, dtype=np.float64)
    return prob_stub


def make_custom(kind: str, n, bounds, nlev, bc, M=0.0, a=0.0,
                recon=RECON_PLM, geo_extent=None) -> Problem:
    """A bare geometry (no fluid randomness) for pins and small tests: rho=1,
    u=0, T=1, kappa=0; callers overwrite fields as needed."""
    n = tuple(n)
    xf = []
    for ax in range(3):
        lo, hi = bounds[ax]
        xf.append(lo + (hi - lo) * np.arange(n[ax] + 1) / n[ax])
    if geo_extent is None:
        geo_extent = (1, 1, 1) if kind == "minkowski_cart" else (n[0], n[1], 1)
    geo = _geometry(kind, xf, n, geo_extent, M, a)
    shp = (n[2], n[1], n[0])
    return Problem(name=kind, n=n, geo_extent=tuple(geo_extent), nlev=nlev,
                   recon=recon, bc=tuple(tuple(b) for b in bc), x_faces=xf,
                   rho=np.ones(shp), u_tet=np.zeros(shp + (3,)), T=np.ones(shp),
                   kappa_a=np.zeros(shp), kappa_s=np.zeros(shp),
                   global_n=n, **geo)
