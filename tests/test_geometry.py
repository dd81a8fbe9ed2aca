"""Pins of the oracle's geometry factors (paper Sec. 2.1-2.2).

* tetrad orthonormality g e e = eta and the normal time leg -alpha g^{0a};
* Ricci rotation coefficients: antisymmetric in their first two (lowered)
  indices; zero for the Cartesian identity tetrad of flat space (Sec. 2.2);
  equal to the textbook connection of the orthonormal spherical frame of flat
  space (nabla_theta e_theta = -e_r / r, ...);
* the sphere velocity W used for angular fluxes reproduces the paper's
  n^zeta and n^psi formulas (bracket without 1/2) component by component;
* W equals d n^/d lambda of null geodesics integrated by RK4 from the
  Christoffel symbols and projected onto the tetrad along the path, a route
  that never forms omega.
"""
import math

import numpy as np
import pytest

from oracle import geometry as G
from paper_2302_04283_amd import workloads as W


def _ks_point(r, th, M=1.0, a=0.9):
    gfn = W._metric_kerr_schild_sph(M, a)

    def efn(x1, x2, x3):
        return W.normal_tetrad(gfn(x1, x2, x3))

    x = (np.array([[[r]]]), np.array([[[th]]]), np.array([[[0.3]]]))
    g, dg = W._with_derivs(gfn, *x, [0, 1])
    e, de = W._with_derivs(efn, *x, [0, 1])
    return g[0, 0, 0], dg[0, 0, 0], e[0, 0, 0], de[0, 0, 0], gfn, efn


@pytest.mark.parametrize("r,th", [(1.3, 0.4), (2.0, math.pi / 2), (7.5, 2.9), (40.0, 1.1)])
def test_tetrad(r, th):
    g, _, e, _, _, _ = _ks_point(r, th)
    eta = np.einsum("ma,mn,nb->ab", e, g, e)
    assert np.abs(eta - G.ETA).max() <= 1e-13
    ginv = np.linalg.inv(g)
    alpha = 1.0 / math.sqrt(-ginv[0, 0])
    assert np.abs(e[:, 0] + alpha * ginv[0, :]).max() <= 1e-13


@pytest.mark.parametrize("r,th", [(1.3, 0.4), (2.0, math.pi / 2), (7.5, 2.9)])
def test_omega_antisymmetric(r, th):
    g, dg, e, de, _, _ = _ks_point(r, th)
    om = G.ricci_rotation(g, dg, e, de)
    low = G.lower_omega(om)
    assert np.abs(low + np.swapaxes(low, 0, 1)).max() <= 1e-12 * max(1.0, np.abs(low).max())
    assert np.abs(low).max() > 1e-3     # curved space: non-trivial


def test_omega_zero_cartesian():
    p = W.make_problem("c1")
    om = G.ricci_rotation(p.gcov_c, p.dgcov_c, p.tet_c, p.dtet_c)
    assert np.abs(om).max() == 0.0


@pytest.mark.parametrize("r,th", [(1.7, 0.6), (3.0, 1.9)])
def test_omega_flat_spherical_textbook(r, th):
    g, dg, e, de, _, _ = _ks_point(r, th, M=0.0, a=0.0)
    om = G.ricci_rotation(g, dg, e, de)       # om[c, a, b]: nabla_b e_a, component c
    R, TH, PH = 1, 2, 3
    expect = np.zeros((4, 4, 4))
    expect[R, TH, TH] = -1.0 / r                  # nabla_th e_th = -e_r/r
    expect[TH, R, TH] = 1.0 / r                   # nabla_th e_r  =  e_th/r
    expect[PH, R, PH] = 1.0 / r                   # nabla_ph e_r  =  e_ph/r
    expect[PH, TH, PH] = 1.0 / (r * math.tan(th))  # nabla_ph e_th = cot e_ph/r
    expect[R, PH, PH] = -1.0 / r                  # nabla_ph e_ph = -(e_r + cot e_th)/r
    expect[TH, PH, PH] = -1.0 / (r * math.tan(th))
    assert np.abs(om - expect).max() <= 1e-13


def _random_dirs(n, seed=5):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_sphere_velocity_matches_paper_angle_rates():
    g, dg, e, de, _, _ = _ks_point(2.3, 1.0)
    om = G.ricci_rotation(g, dg, e, de)
    n = _random_dirs(64)
    Wv = G.sphere_velocity(om, n)
    zeta = np.arccos(n[:, 2])
    psi = np.arctan2(n[:, 1], n[:, 0])
    sz = np.sin(zeta)
    n4 = np.concatenate([np.ones((64, 1)), n], 1)
    q = np.einsum("cab,ka,kb->kc", om, n4, n4)
    # paper: n^zeta = sin^-1 n n n^[0 omega^3],  n^psi = sin^-2 n n n^[2 omega^1]
    nzeta = (1.0 * q[:, 3] - n4[:, 3] * q[:, 0]) / sz
    npsi = (n4[:, 2] * q[:, 1] - n4[:, 1] * q[:, 2]) / sz ** 2
    e_zeta = np.stack([np.cos(zeta) * np.cos(psi), np.cos(zeta) * np.sin(psi), -sz], 1)
    e_psi = np.stack([-np.sin(psi), np.cos(psi), np.zeros(64)], 1)
    assert np.abs(np.einsum("ki,ki->k", Wv, e_zeta) - nzeta).max() <= 1e-12
    assert np.abs(np.einsum("ki,ki->k", Wv, e_psi) - sz * npsi).max() <= 1e-12
    assert np.abs(np.einsum("ki,ki->k", Wv, n)).max() <= 1e-12   # tangent


def _christoffel_at(gfn, x):
    xs = tuple(np.array([[[v]]]) for v in x[1:])
    g, dg = W._with_derivs(gfn, *xs, [0, 1])
    return G.christoffel(g[0, 0, 0], dg[0, 0, 0])


def _rk4(gfn, x, k, h):
    def f(x, k):
        Gm = _christoffel_at(gfn, x)
        return k, -np.einsum("mab,a,b->m", Gm, k, k)

    k1x, k1k = f(x, k)
    k2x, k2k = f(x + 0.5 * h * k1x, k + 0.5 * h * k1k)
    k3x, k3k = f(x + 0.5 * h * k2x, k + 0.5 * h * k2k)
    k4x, k4k = f(x + h * k3x, k + h * k3k)
    return (x + h / 6 * (k1x + 2 * k2x + 2 * k3x + k4x),
            k + h / 6 * (k1k + 2 * k2k + 2 * k3k + k4k))


@pytest.mark.parametrize("r,th", [(2.2, 1.2), (6.0, 0.7), (1.45, 1.6)])
def test_sphere_velocity_from_null_geodesics(r, th):
    g, dg, e, de, gfn, efn = _ks_point(r, th)
    om = G.ricci_rotation(g, dg, e, de)
    dirs = _random_dirs(6, seed=int(r * 100))
    Wv = G.sphere_velocity(om, dirs)
    h = 1e-4
    x0 = np.array([0.0, r, th, 0.3])
    for m, nh in enumerate(dirs):
        k0 = e @ np.concatenate([[1.0], nh])       # k^mu = e^mu_b n^b, nu = 1
        nhs = []
        for s in (+1, -1):
            x1, k1 = _rk4(gfn, x0, k0, s * h)
            ee = np.real(efn(*(np.array([[[v]]]) + 0j for v in x1[1:])))[0, 0, 0]
            gg = np.real(gfn(*(np.array([[[v]]]) + 0j for v in x1[1:])))[0, 0, 0]
            kt = G.inverse_tetrad(gg, ee) @ k1     # tetrad components
            nhs.append(kt[1:] / kt[0])
        dn = (nhs[0] - nhs[1]) / (2 * h)
        assert np.abs(dn - Wv[m]).max() <= 1e-6 * max(1.0, np.abs(Wv[m]).max())
