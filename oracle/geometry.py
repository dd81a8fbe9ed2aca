"""Geometry factors of the finite-solid-angle scheme (paper Sec. 2.1-2.2).

Everything is computed once from the problem's metric g_{ab}, its spatial
derivatives, the tetrad e^a_{b^} and its derivatives (stationary spacetime and
tetrad, so d_0 of all of them vanishes):

* Christoffel symbols Gamma^m_{nl} = 1/2 g^{ms}(d_n g_{sl} + d_l g_{sn} - d_s g_{nl});
* Ricci rotation coefficients (Sec. 2.2)
      omega^{c^}_{a^ b^} = e^{c^}_e  e^d_{b^}  nabla_d e^e_{a^},
  with e^{c^}_e = eta^{c^ s^} g_{e m} e^m_{s^};
* per direction n^ (unit 3-vector, n^{0^} = 1): n^a = e^a_{b^} n^{b^} and
  n_a = g_{ab} n^b;
* the tetrad-frame angular velocity on the unit sphere,
      W^i(n^) = -omega^{i}(n,n) + n^i omega^{0}(n,n),
      omega^{c}(n,n) = omega^{c^}_{a^ b^} n^{a^} n^{b^}.
  Its spherical components are the paper's n^zeta and sin(zeta) n^psi (the
  bracket there carries no 1/2, Sec. 1); a test checks that identity and that
  W is tangent to the sphere.

Pins: tests/test_geometry.py (tetrad orthonormality, antisymmetry of omega,
omega = 0 for the Cartesian identity tetrad, the textbook spherical-frame
connection, agreement of W with null geodesics integrated from the
Christoffel symbols).
"""
from __future__ import annotations

import numpy as np

ETA = np.diag([-1.0, 1.0, 1.0, 1.0])


def full_derivative(d_spatial: np.ndarray) -> np.ndarray:
    """[..., 3, 4, 4] spatial derivatives -> [..., 4, 4, 4] with d_0 = 0."""
    out = np.zeros(d_spatial.shape[:-3] + (4,) + d_spatial.shape[-2:])
    out[..., 1:, :, :] = d_spatial
    return out


def christoffel(g: np.ndarray, dg_spatial: np.ndarray) -> np.ndarray:
    """Gamma[..., m, n, l] = Gamma^m_{nl}."""
    dg = full_derivative(dg_spatial)            # dg[..., d, a, b] = d_d g_ab
    ginv = np.linalg.inv(g)
    # lowered: Gamma_{s n l} = 1/2 (d_n g_{s l} + d_l g_{s n} - d_s g_{n l})
    low = 0.5 * (np.einsum("...nsl->...snl", dg) + np.einsum("...lsn->...snl", dg)
                 - dg)
    return np.einsum("...ms,...snl->...mnl", ginv, low)


def inverse_tetrad(g: np.ndarray, e: np.ndarray) -> np.ndarray:
    """einv[..., c^, m] = e^{c^}_m = eta^{c^ s^} g_{m n} e^n_{s^}."""
    return np.einsum("cs,...mn,...ns->...cm", ETA, g, e)


def ricci_rotation(g, dg_spatial, e, de_spatial) -> np.ndarray:
    """omega[..., c, a, b] = omega^{c^}_{a^ b^}."""
    Gam = christoffel(g, dg_spatial)
    de = full_derivative(de_spatial)            # de[..., d, m, a^] = d_d e^m_{a^}
    # nabla_d e^m_{a^} = d_d e^m_{a^} + Gamma^m_{d l} e^l_{a^}
    nab = de + np.einsum("...mdl,...la->...dma", Gam, e)
    einv = inverse_tetrad(g, e)
    return np.einsum("...cm,...db,...dma->...cab", einv, e, nab)


def lower_omega(om: np.ndarray) -> np.ndarray:
    """omega_{c^ a^ b^} = eta_{c^ s^} omega^{s^}_{a^ b^}."""
    return np.einsum("cs,...sab->...cab", ETA, om)


def four_dir(nhat: np.ndarray) -> np.ndarray:
    """n^{a^} = (1, n^) for unit 3-vectors [..., 3] -> [..., 4]."""
    return np.concatenate([np.ones(nhat.shape[:-1] + (1,)), nhat], axis=-1)


def n_up(e: np.ndarray, nhat: np.ndarray) -> np.ndarray:
    """n^a for every geometry point x direction: [G..., N, 4]."""
    return np.einsum("...mb,nb->...nm", e, four_dir(nhat))


def n_down(g: np.ndarray, e: np.ndarray, nhat: np.ndarray) -> np.ndarray:
    """n_a = g_{ab} n^b: [G..., N, 4]."""
    return np.einsum("...am,...nm->...na", g, n_up(e, nhat))


def sphere_velocity(om: np.ndarray, mhat: np.ndarray) -> np.ndarray:
    """W(m^) = -omega^i(m,m) + m^i omega^0(m,m): [G..., M, 3]."""
    m4 = four_dir(mhat)
    q = np.einsum("...cab,ka,kb->...kc", om, m4, m4)      # omega^c(m,m)
    return -q[..., 1:] + mhat * q[..., :1]
