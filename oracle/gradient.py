"""Reference gradient of the outgoing-luminosity functional (test infrastructure).

J = sum over steps of dt * l(I_s): the energy the scheme moves out through the
luminosity face during the run (l as in ``step.transport``).  Its gradient
with respect to the per-cell absorption and scattering opacities, the initial
gas temperature and the initial intensities is obtained by reverse-mode
automatic differentiation through the oracle's own step; the quartic's root
carries the implicit-function backward of ``quartic.py``.  Each step can be
recomputed during the backward pass (``checkpoint=True``) to bound memory.

Pins: tests/test_oracle_gradient.py compares it with central finite
differences of the oracle's J.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint as _ckpt

from . import step as O


def functional(prob, S, I0, T0, dt, nsteps, kappa_a=None, kappa_s=None, checkpoint=False):
    """J for the given (differentiable) inputs."""
    rho, u, ka0, ks0 = O.fluid_tensors(prob)
    ka = ka0 if kappa_a is None else kappa_a
    ks = ks0 if kappa_s is None else kappa_s
    ba = O.beam_angle(S) if prob.beam_mask is not None else None
    I, T = I0, T0
    J = torch.zeros((), dtype=torch.float64)

    def one(I, T, ka, ks):
        Ip, Tp, _, dl = O.step(I, T, S, rho, u, ka, ks, dt, ba)
        return Ip, Tp, dl

    for _ in range(nsteps):
        if checkpoint:
            I, T, dl = _ckpt(one, I, T, ka, ks, use_reentrant=False)
        else:
            I, T, dl = one(I, T, ka, ks)
        J = J + dl
    return J


def reference_gradient(prob, I0, T0, dt, nsteps, checkpoint=False):
    """Returns dict(J, kappa_a, kappa_s, T0, I0) with gradients of J."""
    S = O.setup(prob)
    ka = torch.as_tensor(prob.kappa_a).clone().requires_grad_(True)
    ks = torch.as_tensor(prob.kappa_s).clone().requires_grad_(True)
    T = torch.as_tensor(T0, dtype=torch.float64).clone().requires_grad_(True)
    I = torch.as_tensor(I0, dtype=torch.float64).clone().requires_grad_(True)
    J = functional(prob, S, I, T, dt, nsteps, ka, ks, checkpoint)
    J.backward()
    return {"J": float(J.detach()), "kappa_a": ka.grad.numpy(), "kappa_s": ks.grad.numpy(),
            "T0": T.grad.numpy(), "I0": I.grad.numpy()}


def functional_value(prob, I0, T0, dt, nsteps):
    """J without gradients (for finite differences)."""
    S = O.setup(prob)
    with torch.no_grad():
        return float(functional(prob, S, torch.as_tensor(I0, dtype=torch.float64),
                                torch.as_tensor(T0, dtype=torch.float64), dt, nsteps))
