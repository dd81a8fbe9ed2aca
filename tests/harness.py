"""Test harness: the same seeded problem through the HIP library and the oracle."""
from __future__ import annotations

import numpy as np
import torch

from oracle import step as O
from paper_2302_04283_amd import rt


def gpu_run(prob, precision, steps, dt, I0=None, T0=None, device=0, grid=None):
    """Run `steps` library steps; returns host float64 arrays (I, T, dT0, J) and the grid."""
    g = grid or rt.Grid(prob, precision, device)
    dev = torch.device("cuda", device)
    rd = g.real_dtype()
    if I0 is None:
        I0 = prob.initial_intensity()
    Ia = torch.as_tensor(np.ascontiguousarray(I0)).to(dev, rd)
    Ib = torch.empty_like(Ia)
    T = torch.as_tensor(np.ascontiguousarray(prob.T if T0 is None else T0)).to(dev)
    rho = torch.as_tensor(prob.rho).to(dev)
    u = torch.as_tensor(prob.u_tet).to(dev)
    ka = torch.as_tensor(prob.kappa_a).to(dev)
    ks = torch.as_tensor(prob.kappa_s).to(dev)
    dT0 = torch.zeros(T.shape + (4,), dtype=torch.float64, device=dev)
    lum = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(steps):
        g.step(Ia, Ib, T, rho, u, ka, ks, dt, dT0, lum)
        Ia, Ib = Ib, Ia
    torch.cuda.synchronize(dev)
    return (Ia.double().cpu().numpy(), T.cpu().numpy(), dT0.cpu().numpy(),
            float(lum.cpu()[0]), g)


def oracle_run(prob, steps, dt, I0=None, T0=None, stats=None):
    S = O.setup(prob)
    if I0 is None:
        I0 = prob.initial_intensity()
    I, T, dT0, J = O.run(prob, S, I0, prob.T if T0 is None else T0, dt, steps, stats)
    return I.numpy(), T.numpy(), dT0.numpy(), float(J), S


def rel_err(x, ref, floor_frac=1e-3):
    """max |x - ref| / (|ref| + floor_frac * max|ref|)."""
    ref = np.asarray(ref)
    scale = np.abs(ref) + floor_frac * np.abs(ref).max()
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(np.asarray(x) - ref) / scale))
