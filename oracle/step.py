"""One forward step of the gray finite-solid-angle scheme (paper Sec. 2).

Order inside a step follows the paper's task list for one stage (Sec. 2):
ghost fill -> reconstruction -> upwind spatial and angular fluxes -> flux
divergence -> primitives (with the |n_0| mask, Sec. 2.4) -> implicit
radiation-matter coupling (Sec. 2.5) -> four-momentum bookkeeping.  One
forward-Euler transport stage per step (the paper's multi-stage integrator
reduced to its first stage).

Discrete update (gray integral form, Sec. 2.2), conserved Q = n^0 n_0 I per
(cell c, angle n):

  Q*_{c,n} = Q_{c,n} - dt/dV_c sum_a [dA n^a n_0 I_up]_{c-1/2}^{c+1/2}
                     - dt/dOmega_n sum_{edges e of n} sigma_{n,e} F_{c,e}

  spatial upwind (Sec. 2.4): I_up = I_L if n^a > 0, I_R if n^a < 0, else 0;
  I_L, I_R from donor-cell or van Leer PLM per angle (Sec. 2.3);
  angular flux through edge e = (lo, hi) of the geodesic grid (Sec. 2.6):
  F_e = L_e (W(m_e) . nu_e) n_0(m_e) I_up, I_up = I_lo if W.nu > 0,
  I_hi if W.nu < 0; sigma = +1 for lo, -1 for hi.

Then I* = Q*/(n^0 n_0), zeroed where |n_0| < n0_crit.

Coupling per cell (Sec. 2.5), with fluid-frame quantities from the boost
n^0bar = u^0^ - u^.n^ (I_bar = I n0bar^4, dOmega_bar = dOmega/n0bar^2):
  d_n = n^0 + n0bar_n alpha_E dt,  k_n = n^0 / d_n
  E-   = sum_n I*_n n0bar_n^2 dOmega_n
  A1   = sum_n k_n I*_n n0bar_n^2 dOmega_n
  A2   = dt/(4 pi) sum_n dOmega_n / (n0bar_n d_n)
  B4 = A2 alpha_a a_rad,  B1 = rho c_v (1 - A2 alpha_s),
  B0 = A1 - B1 T- - (1 - A2 alpha_s) E-
  T+ = root,  E+ = E- - rho c_v (T+ - T-),  S = alpha_a a_rad T+^4 + alpha_s E+
  I+_n = k_n I*_n + dt S / (4 pi d_n n0bar_n^3)
  dT0_a -= sum_n n^0 n_a (I+_n - I*_n) dOmega_n.

Readings where the paper leaves a choice: masked bins carry zero intensity through the
coupling and are left out of its angle sums; the fixed beam cells are
re-imposed after the coupling; the luminosity is the energy flux the scheme
itself moves through the chosen boundary face.

Optional parts of the scheme (Sec. 2, flux calculation; Sec. 3, diffusion):

  optical-depth-aware flux: per face an optical depth
  tau = C_tau alpha_E dt / u^0^ from the face averages of the two adjacent
  cells' alpha_E = (kappa_a + kappa_s) rho and u^0^, f = -expm1(-tau^2),
  g_L/R = -f (1 + 1/n0bar_L/R) from each cell's own fluid, g = (g_L + g_R)/2,
  and the upwind value times (1 - g_up + g); ghost cells carry the fluid of
  the cell they copy (outflow) or wrap to (periodic).

  two-stage integrator (Heun): stage 1 is the forward-Euler step U1 = U0 +
  dt L(U0) with the coupling over dt; stage 2 forms ((U0 + U1) + dt L(U1))/2
  for the radiation and (T0 + T1)/2 for the gas and applies the coupling over
  dt/2.  The source, the T^0_alpha bookkeeping and the luminosity then enter
  as (S1/2 + S2) and dt (l(U0) + l(U1))/2.

  radiation-dominated velocity substitute (Sec. 2.5): see
  ``radiation_velocity``; the rest of the coupling is unchanged.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import angular_grid as AG
from . import geometry as GEO
from .quartic import quartic_root, quartic_root_count

FOUR_PI = 4.0 * math.pi
MAPR_TIE = 1e-10
BC_PERIODIC = 0
BC_OUTFLOW_VACUUM = 1


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64)


@dataclass
class Setup:
    prob: object
    ang: AG.AngularGrid
    nhat: torch.Tensor        # [N, 3]
    domega: torch.Tensor      # [N]
    n_up_c: torch.Tensor      # [g2,g1,g0,N,4] n^a at cell centres
    n_dn_c: torch.Tensor      # [g2,g1,g0,N,4] n_a at cell centres
    q: torch.Tensor           # [g2,g1,g0,N]   n^0 n_0
    mask: torch.Tensor        # [g2,g1,g0,N]   bool, |n_0| < n0_crit
    face_na: list             # 3 x [f2,f1,f0,N] n^a at face centres (own axis)
    face_C: list              # 3 x [f2,f1,f0,N] dA n^a n_0
    vol: torch.Tensor         # [g2,g1,g0]
    edge_lo: torch.Tensor     # [E] long
    edge_hi: torch.Tensor     # [E] long
    edge_v: torch.Tensor      # [g2,g1,g0,E] L_e W.nu
    edge_w: torch.Tensor      # [g2,g1,g0,E] L_e W.nu n_0(m_e)
    omega: np.ndarray         # [g2,g1,g0,4,4,4]
    edge_ll: torch.Tensor = None   # [E] PLM stencil beyond lo (latitude-longitude)
    edge_rr: torch.Tensor = None   # [E] PLM stencil beyond hi
    mapr: tuple = None             # MAPR geometry (geodesic grids)


def setup(prob) -> Setup:
    """Derived geometry of the scheme for a problem statement."""
    ll = getattr(prob, "latlong", None)
    ang = AG.build_latlong(*ll) if ll is not None else AG.build(prob.nlev)
    recon_a = getattr(prob, "ang_recon", 0)
    if recon_a == 1 and ang.ll is None:
        raise ValueError("angular PLM needs the latitude-longitude grid")
    if recon_a == 2 and ang.ll is not None:
        raise ValueError("MAPR is the geodesic grid's reconstruction")
    mapr = None
    if recon_a == 2:
        nbr, inv, valid, d_lo, d_hi = AG.mapr_geometry(ang)
        cnt = valid.sum(1)
        nxt = np.array([[(i + 1) % cnt[c] if i < cnt[c] else i for i in range(6)]
                        for c in range(len(cnt))])
        mapr = (torch.as_tensor(nbr), torch.as_tensor(nxt), _t(inv), torch.as_tensor(valid),
                _t(d_lo), _t(d_hi))
    nhat = ang.nhat
    nu_c = GEO.n_up(prob.tet_c, nhat)
    nl_c = GEO.n_down(prob.gcov_c, prob.tet_c, nhat)
    q = nu_c[..., 0] * nl_c[..., 0]
    mask = np.abs(nl_c[..., 0]) < prob.n0_crit
    face_na, face_C = [], []
    for a in range(3):
        nu_f = GEO.n_up(prob.tet_f[a], nhat)
        nl_f = GEO.n_down(prob.gcov_f[a], prob.tet_f[a], nhat)
        na = nu_f[..., a + 1]
        face_na.append(_t(na))
        face_C.append(_t(prob.area[a][..., None] * na * nl_f[..., 0]))
    om = GEO.ricci_rotation(prob.gcov_c, prob.dgcov_c, prob.tet_c, prob.dtet_c)
    W = GEO.sphere_velocity(om, ang.mid)                    # [g..,E,3]
    v = ang.length * np.einsum("...ei,ei->...e", W, ang.nu)
    n0m = GEO.n_down(prob.gcov_c, prob.tet_c, ang.mid)[..., 0]
    w = v * n0m
    return Setup(prob=prob, ang=ang, nhat=_t(nhat), domega=_t(ang.domega),
                 n_up_c=_t(nu_c), n_dn_c=_t(nl_c), q=_t(q), mask=torch.as_tensor(mask),
                 face_na=face_na, face_C=face_C, vol=_t(prob.vol),
                 edge_lo=torch.as_tensor(ang.lo), edge_hi=torch.as_tensor(ang.hi),
                 edge_v=_t(v), edge_w=_t(w), omega=om,
                 edge_ll=None if ang.ll is None else torch.as_tensor(ang.ll),
                 edge_rr=None if ang.rr is None else torch.as_tensor(ang.rr), mapr=mapr)


def beam_angle(S: Setup) -> int:
    """Angle whose direction has the largest x^1 component."""
    return int(torch.argmax(S.nhat[:, 0]))


# ----------------------------------------------------------------------------
# transport
# ----------------------------------------------------------------------------

def _nar(x, d, start, length):
    return x.narrow(d, start, length)


def ghost_pad(I: torch.Tensor, S: Setup, a: int) -> torch.Tensor:
    """I padded by two ghost cells along axis a (tensor dim 2-a).

    periodic: wrapped copies.  outflow/vacuum: for directions leaving the
    domain through the boundary face (n^a < 0 at the lower face, > 0 at the
    upper face) the ghosts copy the adjacent active cell; all other
    directions see zero intensity (vacuum inflow)."""
    prob = S.prob
    d = 2 - a
    n = I.shape[d]
    lo_bc, hi_bc = prob.bc[a]
    na = S.face_na[a]
    nf = na.shape[d]
    if lo_bc == BC_PERIODIC:
        g_lo = [_nar(I, d, n - 2, 1), _nar(I, d, n - 1, 1)]
    else:
        first = _nar(I, d, 0, 1)
        out = _nar(na, d, 0, 1) < 0
        gv = torch.where(out, first, torch.zeros_like(first))
        g_lo = [gv, gv]
    if hi_bc == BC_PERIODIC:
        g_hi = [_nar(I, d, 0, 1), _nar(I, d, 1, 1)]
    else:
        last = _nar(I, d, n - 1, 1)
        out = _nar(na, d, nf - 1, 1) > 0
        gv = torch.where(out, last, torch.zeros_like(last))
        g_hi = [gv, gv]
    return torch.cat(g_lo + [I] + g_hi, dim=d)


def face_states(P: torch.Tensor, d: int, n: int, recon: int):
    """Left/right states at the n+1 faces along dim d of a 2-ghost padded array.

    PLM slope (van Leer 1974, harmonic mean): delta = 2 dm dp/(dm + dp) if
    dm dp > 0 else 0, in index space.  Donor cell: delta = 0."""
    cen = _nar(P, d, 1, n + 2)                       # physical cells -1 .. n
    if recon == 1:
        dm = cen - _nar(P, d, 0, n + 2)
        dp = _nar(P, d, 2, n + 2) - cen
        prod = dm * dp
        pos = prod > 0
        den = torch.where(pos, dm + dp, torch.ones_like(dm))
        delta = torch.where(pos, 2.0 * prod / den, torch.zeros_like(dm))
    else:
        delta = torch.zeros_like(cen)
    IL = _nar(cen, d, 0, n + 1) + 0.5 * _nar(delta, d, 0, n + 1)
    IR = _nar(cen, d, 1, n + 1) - 0.5 * _nar(delta, d, 1, n + 1)
    return IL, IR


def fluid_pad(x: torch.Tensor, S: Setup, a: int) -> torch.Tensor:
    """A per-cell field padded by one ghost cell along axis a: wrapped copies
    on periodic boundaries, the adjacent cell's value on outflow/vacuum ones."""
    prob = S.prob
    d = 2 - a
    n = x.shape[d]
    lo = _nar(x, d, n - 1, 1) if prob.bc[a][0] == BC_PERIODIC else _nar(x, d, 0, 1)
    hi = _nar(x, d, 0, 1) if prob.bc[a][1] == BC_PERIODIC else _nar(x, d, n - 1, 1)
    return torch.cat([lo, x, hi], dim=d)


def tau_factors(S: Setup, a: int, fl, dt: float):
    """Optical-depth-aware flux factors (Sec. 2, flux calculation) at the n+1
    faces along axis a for upwind L and upwind R: (1 - g_L + g, 1 - g_R + g)."""
    rho, u, ka, ks = fl
    d = 2 - a
    n = rho.shape[d]
    aE = (ka + ks) * rho
    u0 = torch.sqrt(1.0 + (u * u).sum(-1))
    nbar = u0[..., None] - torch.einsum("...i,ni->...n", u, S.nhat)
    aEp, u0p = fluid_pad(aE, S, a), fluid_pad(u0, S, a)
    nbp = fluid_pad(nbar, S, a)
    aEf = 0.5 * (_nar(aEp, d, 0, n + 1) + _nar(aEp, d, 1, n + 1))
    u0f = 0.5 * (_nar(u0p, d, 0, n + 1) + _nar(u0p, d, 1, n + 1))
    tau = S.prob.tau_coeff * aEf * dt / u0f
    f = -torch.expm1(-tau * tau)
    gL = -f[..., None] * (1.0 + 1.0 / _nar(nbp, d, 0, n + 1))
    gR = -f[..., None] * (1.0 + 1.0 / _nar(nbp, d, 1, n + 1))
    g = 0.5 * (gL + gR)
    # 1 - g_up + g, written so that it is exactly 1 when g_L = g_R
    return 1.0 + (g - gL), 1.0 + (g - gR)


def spatial_fluxes(I: torch.Tensor, S: Setup, a: int, fl=None, dt: float = 0.0) -> torch.Tensor:
    """Face fluxes dA n^a n_0 I_up along axis a: [.., n+1 along dim 2-a, .., N].
    With tau_coeff > 0 (fluid ``fl`` and dt given) the upwind value carries
    the optical-depth-aware factor."""
    d = 2 - a
    n = I.shape[d]
    P = ghost_pad(I, S, a)
    IL, IR = face_states(P, d, n, S.prob.recon)
    if S.prob.tau_coeff > 0.0 and fl is not None:
        fL, fR = tau_factors(S, a, fl, dt)
        IL, IR = IL * fL, IR * fR
    na = S.face_na[a]
    Iup = torch.where(na > 0, IL, torch.where(na < 0, IR, torch.zeros_like(IL)))
    return S.face_C[a] * Iup


def _van_leer_slope(a, b, c):
    """Harmonic-mean slope of b between neighbours a and c (index space)."""
    dm, dp = b - a, c - b
    prod = dm * dp
    pos = prod > 0
    den = torch.where(pos, dm + dp, torch.ones_like(dm))
    return torch.where(pos, 2.0 * prod / den, torch.zeros_like(dm))


def mapr_candidates(I: torch.Tensor, S: Setup):
    """MAPR candidate planes of every cell-direction (Sec. 2.6): the gradient
    in the tangent plane of the plane through the direction and each pair of
    consecutive neighbours, and its squared norm (inf for padding slots).
    Returns (cand [.., N, 6, 2], n2 [.., N, 6])."""
    nbr, nxt, inv, valid, _, _ = S.mapr
    dI = I[..., nbr] - I[..., None]                          # [.., N, 6]
    dJ = torch.gather(dI, -1, nxt.expand(dI.shape))
    cand = torch.einsum("nikl,...nil->...nik", inv, torch.stack([dI, dJ], -1))
    n2 = torch.where(valid, (cand * cand).sum(-1), torch.full_like(dI, math.inf))
    return cand, n2


def mapr_ambiguous(I: torch.Tensor, S: Setup, band: float) -> torch.Tensor:
    """Cell-directions whose MAPR plane choice a lower precision may take
    differently: a candidate whose gradient differs from the flattest one's
    (by more than 1e-6 of the largest gradient of the direction) has a
    squared norm within a relative ``band`` of the smallest.  bool [.., N]."""
    cand, n2 = mapr_candidates(I, S)
    nmin = n2.min(-1, keepdim=True).values
    near = n2 <= nmin * (1.0 + band)
    k = torch.argmin(n2, -1, keepdim=True)
    best = torch.gather(cand, -2, k[..., None].expand(k.shape + (2,)))
    gmax = torch.sqrt(torch.where(torch.isfinite(n2), n2, torch.zeros_like(n2)).max(-1).values)
    differs = ((cand - best).abs().amax(-1) > 1e-6 * gmax[..., None])
    return (near & differs).any(-1)


def angular_divergence(I: torch.Tensor, S: Setup) -> torch.Tensor:
    """sum over the edges of each angular cell of sigma F_e: [.., N].
    Upwind value: the cell value (DC) or, with angular PLM on the
    latitude-longitude grid (Sec. 2.3), the van Leer face value from the
    stencil (ll, lo, hi, rr) along the edge's coordinate line."""
    lo, hi = S.edge_lo, S.edge_hi
    v, w = S.edge_v, S.edge_w
    Ilo = I[..., lo]
    Ihi = I[..., hi]
    if getattr(S.prob, "ang_recon", 0) == 2:
        # MAPR: per cell-direction the flattest of the candidate planes
        _, _, _, _, d_lo, d_hi = S.mapr
        cand, n2 = mapr_candidates(I, S)
        # the first candidate (in the grid's order) within a relative
        # tolerance of the flattest: ties between equally flat planes, which
        # the grid's symmetry produces, are broken by position, not by
        # rounding
        near = n2 <= n2.min(-1, keepdim=True).values * (1.0 + MAPR_TIE)
        k = torch.argmax(near.to(torch.int8), -1, keepdim=True)
        grad = torch.gather(cand, -2, k[..., None].expand(k.shape + (2,))).squeeze(-2)
        Ilo = Ilo + (grad[..., lo, :] * d_lo).sum(-1)
        Ihi = Ihi + (grad[..., hi, :] * d_hi).sum(-1)
    elif getattr(S.prob, "ang_recon", 0):
        Ill = I[..., S.edge_ll]
        Irr = I[..., S.edge_rr]
        IL = Ilo + 0.5 * _van_leer_slope(Ill, Ilo, Ihi)
        IR = Ihi - 0.5 * _van_leer_slope(Ilo, Ihi, Irr)
        Ilo, Ihi = IL, IR
    Iup = torch.where(v > 0, Ilo, torch.where(v < 0, Ihi, torch.zeros_like(Ilo)))
    F = w * Iup
    div = torch.zeros_like(I)
    div = div.index_add(I.dim() - 1, lo, F)
    div = div.index_add(I.dim() - 1, hi, -F)
    return div


def transport(I: torch.Tensor, S: Setup, dt: float, stats: dict | None = None, fl=None,
              base=None):
    """Flux divergence and primitive recovery: returns (I*, luminosity rate).

    The luminosity rate is the energy per unit time leaving through the
    boundary face (lum_axis, lum_side): minus the sum over that face's fluxes
    weighted by solid angle, with the sign of the outward normal.
    ``base`` = I0 makes this the second stage of the two-stage integrator:
    Q* = (q I0 + q I - dt div(I)) / 2 (``dt`` is then the full step)."""
    prob = S.prob
    Q = S.q * I
    dQ = torch.zeros_like(I)
    lum_rate = torch.zeros((), dtype=I.dtype)
    for a in range(3):
        d = 2 - a
        n = I.shape[d]
        F = spatial_fluxes(I, S, a, fl, dt)
        dQ = dQ + (_nar(F, d, 1, n) - _nar(F, d, 0, n))
        if a == prob.lum_axis:
            f = n if prob.lum_side == 1 else 0
            sgn = 1.0 if prob.lum_side == 1 else -1.0
            Ff = _nar(F, d, f, 1)
            lum_rate = -sgn * torch.sum(Ff * S.domega)
    Qs = Q - dt * dQ / S.vol[..., None] - dt * angular_divergence(I, S) / S.domega
    if base is not None:
        Qs = 0.5 * (S.q * base + Qs)
    Is = Qs / S.q
    if stats is not None:
        # the two-stage step keeps half of stage 1's update (S1/2 + S2)
        wgt = 0.5 if (prob.integrator == 2 and base is None) else 1.0
        removed = -(S.vol[..., None] * S.domega * Qs * S.mask).sum()
        stats["masked_energy"] = stats.get("masked_energy", 0.0) + float(removed) * wgt
    Is = torch.where(S.mask, torch.zeros_like(Is), Is)
    return Is, lum_rate


# ----------------------------------------------------------------------------
# coupling
# ----------------------------------------------------------------------------

def radiation_velocity(Is: torch.Tensor, T: torch.Tensor, S: Setup, rho, u, ka, ks, dt):
    """Velocity used by the coupling in radiation-dominated cells (Sec. 2.5).

    With the gas velocity u: E- = sum I* n0bar^2 dOmega; a cell is radiation
    dominated when E- > rho + u_gas.  There the tetrad-frame moments
    R^00 = sum I* dOmega, R^0a = sum n^a I* dOmega give v_rad = R^0a / R^00
    and u_rad; the force on the gas is
      G^a = -(alpha_a a_rad T^4 + alpha_s E-) u^a - alpha_E u_b R^ab,
      u_b R^ab = -sum n^a n0bar I* dOmega,
    the momentum densities T_gas^0a = w u^0 u^a, T_rad^0a = w u_rad^0 u_rad^a
    (w = rho + u_gas + p), and the fraction per axis
      f^a = clamp(G^a dt / (n^0 (T_rad^0a - T_gas^0a)), 0, 1)
    blends u^a -> (1 - f^a) u^a + f^a u_rad^a.  Other cells (and cells with
    R^00 <= 0 or |v_rad| >= 1) keep u.  Masked bins are left out of the sums.

    The factor n^0 = 1/alpha (the normal observer's n^0, Sec. 2.2): the
    coupling's operator-split momentum equation d_0 T^0_alpha = G_alpha with a
    stationary tetrad makes the gas's tetrad-frame momentum change by
    G^a dt / n^0 over a coordinate step dt (the coupling's own implicit
    factors run over the same dt / n^0), so f^a is the share of the gap
    T_rad^0a - T_gas^0a that one step of the force closes.  (The printed
    divisor u^a is singular for gas at rest and changes sign with the
    direction of motion; see the design notes.)"""
    prob = S.prob
    cv = prob.kb_mu_mp / (prob.gamma_gas - 1.0)
    u0 = torch.sqrt(1.0 + (u * u).sum(-1))
    nbar = u0[..., None] - torch.einsum("...i,ni->...n", u, S.nhat)
    dOm = S.domega * (~S.mask)
    Em = (Is * nbar * nbar * dOm).sum(-1)
    R00 = (Is * dOm).sum(-1)
    R0a = torch.einsum("...n,na->...a", Is * dOm, S.nhat)
    uR = -torch.einsum("...n,na->...a", Is * nbar * dOm, S.nhat)
    ugas = rho * cv * T
    pgas = rho * prob.kb_mu_mp * T
    w = rho + ugas + pgas
    aa, as_ = ka * rho, ks * rho
    safe = R00 > 0.0
    v = torch.where(safe[..., None], R0a / torch.where(safe, R00, torch.ones_like(R00))[..., None],
                    torch.zeros_like(R0a))
    v2 = (v * v).sum(-1)
    ok = safe & (v2 < 1.0) & (Em > rho + ugas)
    ur0 = 1.0 / torch.sqrt(torch.where(ok, 1.0 - v2, torch.ones_like(v2)))
    ur = ur0[..., None] * v
    G = (-(aa * prob.a_rad * T ** 4 + as_ * Em)[..., None] * u - (aa + as_)[..., None] * uR)
    gap = (w * ur0)[..., None] * ur - (w * u0)[..., None] * u
    n0 = S.n_up_c[..., 0, 0]                    # e^0_0^, the same for every direction
    den = n0[..., None] * gap
    f = torch.where(den != 0.0, G * dt / torch.where(den != 0.0, den, torch.ones_like(den)),
                    torch.zeros_like(den)).clamp(0.0, 1.0)
    us = (1.0 - f) * u + f * ur
    return torch.where(ok[..., None], us, u)


def coupling(Is: torch.Tensor, T: torch.Tensor, S: Setup, rho, u, ka, ks, dt,
             stats: dict | None = None):
    """Implicit radiation-matter coupling (Sec. 2.5).  Returns (I+, T+, dT0).
    With rad_velocity set, radiation-dominated cells couple at the velocity
    of ``radiation_velocity`` instead of the gas velocity."""
    prob = S.prob
    cv = prob.kb_mu_mp / (prob.gamma_gas - 1.0)
    if getattr(prob, "rad_velocity", 0):
        u = radiation_velocity(Is, T, S, rho, u, ka, ks, dt)
    u0 = torch.sqrt(1.0 + (u * u).sum(-1))                        # [cells]
    nbar = u0[..., None] - torch.einsum("...i,ni->...n", u, S.nhat)  # [cells, N]
    n0 = S.n_up_c[..., 0]                                          # n^0
    aa = ka * rho
    as_ = ks * rho
    aE = aa + as_
    dOm = S.domega * (~S.mask)                                     # masked bins left out
    dn = n0 + nbar * aE[..., None] * dt
    k = n0 / dn
    w2 = nbar * nbar * dOm
    Em = (Is * w2).sum(-1)
    A1 = (k * Is * w2).sum(-1)
    A2 = dt / FOUR_PI * (dOm / (nbar * dn)).sum(-1)
    B4 = A2 * aa * prob.a_rad
    B1 = rho * cv * (1.0 - A2 * as_)
    B0 = A1 - B1 * T - (1.0 - A2 * as_) * Em
    Tp = quartic_root(B4, B1, B0)
    if stats is not None:
        _, nbad = quartic_root_count(B4.detach(), B1.detach(), B0.detach())
        stats["no_root"] = stats.get("no_root", 0) + nbad
    Ep = Em - rho * cv * (Tp - T)
    Ssrc = aa * prob.a_rad * Tp ** 4 + as_ * Ep
    Ip = k * Is + dt * Ssrc[..., None] / (FOUR_PI * dn * nbar ** 3)
    Ip = torch.where(S.mask, torch.zeros_like(Ip), Ip)
    dI = (Ip - Is) * S.domega
    dT0 = -torch.einsum("...n,...na->...a", n0 * dI, S.n_dn_c)
    return Ip, Tp, dT0


def _impose_beam(Ip, S: Setup, beam_angle_idx):
    prob = S.prob
    if prob.beam_mask is not None and beam_angle_idx is not None:
        bm = torch.as_tensor(prob.beam_mask)
        sel = torch.zeros_like(Ip, dtype=torch.bool)
        sel[..., beam_angle_idx] = bm
        Ip = torch.where(sel, torch.full_like(Ip, prob.beam_I), Ip)
    return Ip


def step(I, T, S: Setup, rho, u, ka, ks, dt, beam_angle_idx=None,
         stats: dict | None = None):
    """One full step.  Returns (I+, T+, dT0 increment, dt * luminosity rate)."""
    fl = (rho, u, ka, ks)
    Is, lum_rate = transport(I, S, dt, stats, fl)
    Ip, Tp, dT0 = coupling(Is, T, S, rho, u, ka, ks, dt, stats)
    Ip = _impose_beam(Ip, S, beam_angle_idx)
    if S.prob.integrator != 2:
        return Ip, Tp, dT0, dt * lum_rate
    # second stage of the two-stage integrator
    Is2, lum_rate2 = transport(Ip, S, dt, stats, fl, base=I)
    Ip2, Tp2, dT02 = coupling(Is2, 0.5 * (T + Tp), S, rho, u, ka, ks, 0.5 * dt, stats)
    Ip2 = _impose_beam(Ip2, S, beam_angle_idx)
    return Ip2, Tp2, 0.5 * dT0 + dT02, 0.5 * dt * (lum_rate + lum_rate2)


def fluid_tensors(prob):
    return (_t(prob.rho), _t(prob.u_tet), _t(prob.kappa_a), _t(prob.kappa_s))


def run(prob, S: Setup, I0, T0, dt, nsteps, stats=None):
    """Run ``nsteps`` steps from (I0, T0).  Returns (I, T, dT0 sum, J)."""
    rho, u, ka, ks = fluid_tensors(prob)
    I = _t(I0)
    T = _t(T0)
    dT0 = torch.zeros(T.shape + (4,), dtype=torch.float64)
    J = torch.zeros((), dtype=torch.float64)
    ba = beam_angle(S) if prob.beam_mask is not None else None
    for _ in range(nsteps):
        I, T, d0, dl = step(I, T, S, rho, u, ka, ks, dt, ba, stats)
        dT0 = dT0 + d0
        J = J + dl
    return I, T, dT0, J


# ----------------------------------------------------------------------------
# moments and time step
# ----------------------------------------------------------------------------
RT_PAIRS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


def moments(I, S: Setup, u):
    """Per-cell R^{a^ b^} = sum I n^a^ n^b^ dOmega (10, upper triangle),
    R^0_a = sum n^0 n_a I dOmega (4), E_fluid = sum I n0bar^2 dOmega."""
    n4 = torch.cat([torch.ones(S.nhat.shape[0], 1, dtype=torch.float64), S.nhat], -1)
    Iw = I * S.domega
    R = torch.stack([(Iw * n4[:, a] * n4[:, b]).sum(-1) for a, b in RT_PAIRS], -1)
    R0 = torch.einsum("...n,...na->...a", S.n_up_c[..., 0] * Iw, S.n_dn_c)
    u0 = torch.sqrt(1.0 + (u * u).sum(-1))
    nbar = u0[..., None] - torch.einsum("...i,ni->...n", u, S.nhat)
    E = (Iw * nbar * nbar).sum(-1)
    return R, R0, E


def max_dt(S: Setup, cfl: float) -> float:
    """dt = cfl * min over cells and angles of
    min( min_a dx^a n^0/|n^a| , dOmega_n n^0 / sum_{outflow edges} |v| ).
    parity unpinned (a time-step rule is a specification, not physics)."""
    prob = S.prob
    n0 = S.n_up_c[..., 0]
    best = float("inf")
    for a in range(3):
        dx = np.diff(prob.x_faces[a])[: prob.geo_extent[a]]
        shp = [1, 1, 1]
        shp[2 - a] = dx.size
        dxt = _t(dx.reshape(shp))[..., None]
        na = S.n_up_c[..., a + 1].abs()
        r = torch.where(na > 0, dxt * n0 / torch.where(na > 0, na, torch.ones_like(na)),
                        torch.full_like(na, float("inf")))
        best = min(best, float(r.min()))
    v = S.edge_v
    N = S.nhat.shape[0]
    outsum = torch.zeros(v.shape[:-1] + (N,), dtype=torch.float64)
    outsum = outsum.index_add(v.dim() - 1, S.edge_lo, torch.clamp(v, min=0.0))
    outsum = outsum.index_add(v.dim() - 1, S.edge_hi, torch.clamp(-v, min=0.0))
    r = torch.where(outsum > 0, S.domega * n0 / torch.where(outsum > 0, outsum,
                                                            torch.ones_like(outsum)),
                    torch.full_like(outsum, float("inf")))
    best = min(best, float(r.min()))
    return cfl * best
