"""Pins of the oracle's reference gradient (autograd through the oracle's step)
against central finite differences of the oracle's own functional, and of the
quartic's implicit-function backward against torch.autograd.gradcheck."""
import numpy as np
import pytest
import torch

from oracle import gradient as GR
from oracle import step as O
from oracle.quartic import quartic_root
from paper_2302_04283_amd import workloads as W


def test_quartic_backward_gradcheck():
    rng = np.random.default_rng(0)
    B4 = torch.tensor(10.0 ** rng.uniform(-3, 1, 8), dtype=torch.float64, requires_grad=True)
    B1 = torch.tensor(10.0 ** rng.uniform(-1, 1, 8), dtype=torch.float64, requires_grad=True)
    B0 = torch.tensor(-(10.0 ** rng.uniform(-1, 1, 8)), dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(quartic_root, (B4, B1, B0), eps=1e-7, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("cfg,scale,steps", [("c4", (8, 6, 4), 6), ("c2", (8, 8, 8), 4)])
def test_reference_gradient_vs_finite_differences(cfg, scale, steps):
    p = W.make_problem(cfg, scale=scale)
    if cfg == "c2":
        p.lum_axis, p.lum_side = 0, 1
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    I0 = p.initial_intensity()
    T0 = p.T.copy()
    g = GR.reference_gradient(p, I0, T0, dt, steps)
    for key in ("kappa_a", "kappa_s", "T0"):
        G = g[key]
        top = np.argsort(-np.abs(G).ravel())[:3]
        for flat in top:
            c = np.unravel_index(flat, G.shape)

            def J_at(sign):
                q = W.make_problem(cfg, scale=scale)
                q.lum_axis, q.lum_side = p.lum_axis, p.lum_side
                T = T0.copy()
                if key == "kappa_a":
                    h = 1e-6 * q.kappa_a[c]
                    q.kappa_a[c] += sign * h
                elif key == "kappa_s":
                    h = 1e-6 * q.kappa_s[c]
                    q.kappa_s[c] += sign * h
                else:
                    h = 1e-6 * T[c]
                    T[c] += sign * h
                return GR.functional_value(q, I0, T, dt, steps), h

            jp, h = J_at(+1)
            jm, _ = J_at(-1)
            fd = (jp - jm) / (2 * h)
            assert abs(G[c] - fd) <= 1e-4 * abs(fd) + 1e-12 * abs(g["J"]) / h, (key, c, G[c], fd)
