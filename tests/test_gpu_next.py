"""The two-stage integrator and the optical-depth-aware flux (general kernel)
against the oracle, through the C ABI.

Tolerances as in test_gpu_parity.py: FP64 intensities 1e-12 and gas
temperature 1e-13 (summation order only); FP32 intensities 1e-5 and gas
temperature 2e-7.
"""
import numpy as np
import pytest
import torch

from harness import gpu_run, oracle_run, rel_err
from oracle import step as O
from paper_2302_04283_amd import rt
from paper_2302_04283_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problem(kind, integrator, tau):
    if kind == "mink":
        p = W.make_problem("c2", scale=(8, 6, 5), nlev=2)
    else:
        p = W.make_problem("c3", scale=(10, 8, 4), nlev=2)
    p.integrator = integrator
    p.tau_coeff = tau
    return p


@pytest.mark.parametrize("prec", [rt.RT_F64, rt.RT_F32])
@pytest.mark.parametrize("kind,integrator,tau", [("mink", 2, 0.0), ("mink", 1, 5.0), ("mink", 2, 5.0),
                                                 ("ks", 2, 0.0), ("ks", 1, 3.0), ("ks", 2, 3.0)])
def test_two_stage_and_tau_flux_match_oracle(kind, integrator, tau, prec):
    p = _problem(kind, integrator, tau)
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    stats = {}
    Io, To, dTo, Jo, _ = oracle_run(p, 3, dt, stats=stats)
    Ig, Tg, dTg, Jg, g = gpu_run(p, prec, 3, dt)
    assert not g.fast_path
    st = g.stats()
    g.close()
    eI = rel_err(Ig, Io)
    eT = float(np.max(np.abs(Tg - To) / To))
    edT = float(np.max(np.abs(dTg - dTo)) / max(np.abs(dTo).max(), 1e-300))
    eJ = abs(Jg - Jo) / max(abs(Jo), 1e-300)
    print("[next] %s integrator=%d tau=%g %s e_I=%.2e e_T=%.2e e_dT0=%.2e e_J=%.2e" % (
        kind, integrator, tau, "fp64" if prec == rt.RT_F64 else "fp32", eI, eT, edT, eJ), flush=True)
    if prec == rt.RT_F64:
        assert eI <= 1e-12 and eT <= 1e-13 and edT <= 1e-12 and eJ <= 1e-12
        assert st["no_root"] == stats.get("no_root", 0)
        me_o = stats.get("masked_energy", 0.0)
        assert abs(st["masked_energy"] - me_o) <= 1e-12 * max(abs(me_o), 1e-300)
    else:
        assert eI <= 1e-5 and eT <= 2e-7


def test_options_select_general_kernel_and_exclude_adjoint():
    p = _problem("mink", 2, 0.0)
    p2 = W.make_problem("c2", scale=(8, 8, 8))
    g0 = rt.Grid(p2, rt.RT_F64)
    assert g0.fast_path
    g0.close()
    g = rt.Grid(p, rt.RT_F64)
    assert not g.fast_path
    dev = torch.device("cuda", 0)
    shape = (p.n[2], p.n[1], p.n[0], g.nang)
    I = torch.zeros(shape, dtype=torch.float64, device=dev)
    cell = torch.ones(shape[:3], dtype=torch.float64, device=dev)
    u = torch.zeros(shape[:3] + (3,), dtype=torch.float64, device=dev)
    with pytest.raises(rt.RtError):
        g.step(I, I.clone(), cell, cell, u, cell, cell, 0.01, I_star=I.clone())
    with pytest.raises(rt.RtError):
        g.step_adjoint(I, cell, cell, u, cell, cell, 0.01, I.clone(), cell.clone(), I.clone(),
                       cell.clone(), I.clone())
    g.close()


@pytest.mark.parametrize("prec", [rt.RT_F64, rt.RT_F32])
def test_two_stage_on_the_tiled_path_matches_oracle(prec):
    """The two-stage integrator on the tiled kernel (162 directions, 32 lanes
    x 6 directions per lane), with the collimated beam and the luminosity."""
    p = W.make_problem("c2", scale=(8, 8, 8))
    p.integrator = 2
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    stats = {}
    Io, To, dTo, Jo, _ = oracle_run(p, 3, dt, stats=stats)
    Ig, Tg, dTg, Jg, g = gpu_run(p, prec, 3, dt)
    assert g.fast_path
    st = g.stats()
    g.close()
    eI = rel_err(Ig, Io)
    eT = float(np.max(np.abs(Tg - To) / To))
    edT = float(np.max(np.abs(dTg - dTo)) / max(np.abs(dTo).max(), 1e-300))
    eJ = abs(Jg - Jo) / max(abs(Jo), 1e-300)
    print("[next] tiled integrator=2 %s e_I=%.2e e_T=%.2e e_dT0=%.2e e_J=%.2e" % (
        "fp64" if prec == rt.RT_F64 else "fp32", eI, eT, edT, eJ), flush=True)
    if prec == rt.RT_F64:
        assert eI <= 1e-12 and eT <= 1e-13 and edT <= 1e-12 and eJ <= 1e-12
        assert st["no_root"] == stats.get("no_root", 0)
    else:
        assert eI <= 1e-5 and eT <= 2e-7
