"""Handing the coupling's four-momentum to the gas (Sec. 2.5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The coupling keeps total four-momentum by taking the change of the
radiation's R^0_alpha from the gas's T^0_alpha; the step returns that change
as dT0 (coordinate components, covariant index).  For a gamma-law gas without
magnetic fields T^{mu nu} = w u^mu u^nu + p g^{mu nu} with p = rho kb T
(kb = k_B / mu m_p), w = rho + Gamma p / (Gamma - 1), and the coupling leaves
the conserved density rho u^0 unchanged (Sec. 2.5).  ``apply`` takes the gas
state from before the step, adds dT0 to T^0_alpha and recovers the primitive
state:

  T^{0 mu} = T^0_alpha g^{alpha mu};  with a normal-observer tetrad
  (e^{0^}_i = 0, e^0_{a^} = 0 for spatial a^) the tetrad row is
  T^{0^ b^} = e^{0^}_0 e^{b^}_mu T^{0 mu}, and rho u^0 held means
  D = rho u^{0^} held;
  E = T^{0^ 0^}, S^a = T^{0^ a^}: p solves w gamma^2 - p - E = 0 with
  v = |S| / (E + p), gamma = (1 - v^2)^(-1/2), rho = D / gamma, by bisection
  to round-off; then u^{a^} = gamma S^a / (E + p), T = p / (rho kb).

The algebra is the standard special-relativistic conserved-to-primitive
inversion of an ideal gas in the local tetrad frame; it is pinned by a
round trip (dT0 = 0 returns the state) and by the moving-equilibration
system of Sec. 3.
"""
from __future__ import annotations

import numpy as np

from .geometry import inverse_tetrad


def gas_T0(prob, rho, u_tet, T):
    """T^0_alpha of the gas, [cells, 4] (coordinate components)."""
    g = np.asarray(prob.gcov_c)
    e = np.asarray(prob.tet_c)
    kb, gam = prob.kb_mu_mp, prob.gamma_gas
    p = rho * kb * T
    w = rho + gam / (gam - 1.0) * p
    ut = np.concatenate([np.sqrt(1.0 + (u_tet * u_tet).sum(-1))[..., None], u_tet], -1)
    uc = np.einsum("...mb,...b->...m", e, ut)
    ul = np.einsum("...mn,...n->...m", g, uc)
    out = (w * uc[..., 0])[..., None] * ul
    out[..., 0] += p
    return out


def apply(prob, rho, u_tet, T_pre, dT0):
    """Gas state after adding dT0 to T^0_alpha of (rho, u_tet, T_pre), with
    rho u^0 held.  All arrays [n2][n1][n0](...) float64; returns new
    (rho, u_tet, T)."""
    rho = np.asarray(rho, dtype=np.float64)
    u_tet = np.asarray(u_tet, dtype=np.float64)
    T_pre = np.asarray(T_pre, dtype=np.float64)
    g = np.broadcast_to(np.asarray(prob.gcov_c), rho.shape + (4, 4))
    e = np.broadcast_to(np.asarray(prob.tet_c), rho.shape + (4, 4))
    einv = inverse_tetrad(g, e)
    if np.abs(einv[..., 0, 1:]).max() > 1e-12 * np.abs(einv[..., 0, 0]).max() or \
            np.abs(e[..., 0, 1:]).max() > 1e-12 * np.abs(e[..., 0, 0]).max():
        raise ValueError("fluid update needs a normal-observer tetrad")
    kb, gam = prob.kb_mu_mp, prob.gamma_gas
    T0 = gas_T0(prob, rho, u_tet, T_pre) + np.asarray(dT0, dtype=np.float64)
    ginv = np.linalg.inv(g)
    Tup = np.einsum("...a,...am->...m", T0, ginv)                  # T^{0 mu}
    row = einv[..., 0, 0][..., None] * np.einsum("...bm,...m->...b", einv, Tup)
    E = row[..., 0]
    S = row[..., 1:]
    Sm = np.sqrt((S * S).sum(-1))
    D = rho * np.sqrt(1.0 + (u_tet * u_tet).sum(-1))

    def resid(p):
        v = Sm / (E + p)
        gm = 1.0 / np.sqrt(1.0 - v * v)
        r = D / gm
        return (r + gam / (gam - 1.0) * p) * gm * gm - p - E

    if not np.all(E > Sm):
        raise ValueError("gas energy below its momentum")
    lo = np.zeros_like(E)
    if np.any(resid(lo) > 0.0):
        raise ValueError("gas energy below its rest mass and kinetic energy")
    hi = np.maximum(E, 1e-300)
    for _ in range(2000):
        bad = resid(hi) <= 0.0
        if not bad.any():
            break
        hi = np.where(bad, 2.0 * hi, hi)
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        done = (mid <= lo) | (mid >= hi)
        if done.all():
            break
        neg = resid(mid) <= 0.0
        lo = np.where(neg & ~done, mid, lo)
        hi = np.where(~neg & ~done, mid, hi)
    p = 0.5 * (lo + hi)
    v = Sm / (E + p)
    gm = 1.0 / np.sqrt(1.0 - v * v)
    rho_n = D / gm
    u_n = (gm / (E + p))[..., None] * S
    return rho_n, u_n, p / (rho_n * kb)
