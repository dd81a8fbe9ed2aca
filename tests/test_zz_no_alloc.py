"""rt_step_noalloc: the step with its per-block partial sums in the library's
static device scratch gives bit-identical results to rt_step, on two calls
in a row (the second on a smaller grid), and rejects a grid whose partial
sums exceed the scratch before any launch."""
import numpy as np
import pytest
import torch

from paper_2302_04283_amd import rt
from paper_2302_04283_amd import workloads as W

pytestmark = pytest.mark.gpu


def _inputs(prob, g, dev):
    I = torch.as_tensor(prob.initial_intensity()).to(dev, g.real_dtype())
    f = [torch.as_tensor(x).to(dev) for x in (prob.T, prob.rho, prob.u_tet, prob.kappa_a,
                                               prob.kappa_s)]
    return I, f


def _one_step(prob, precision, noalloc, dt):
    dev = torch.device("cuda", 0)
    g = rt.Grid(prob, precision, 0)
    I, (T, rho, u, ka, ks) = _inputs(prob, g, dev)
    out = torch.empty_like(I)
    dT0 = torch.zeros(T.shape + (4,), dtype=torch.float64, device=dev)
    lum = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(2):
        g.step(I, out, T, rho, u, ka, ks, dt, dT0, lum, noalloc=noalloc)
        I, out = out, I
    torch.cuda.synchronize(dev)
    st = g.stats()
    res = (I.cpu(), T.cpu(), dT0.cpu(), lum.cpu(), st["no_root"], st["masked_energy"],
           g.fast_path)
    g.close()
    return res


@pytest.mark.parametrize("case", ["tiled_fp32", "general_fp64", "two_stage_fp32", "column_fp32"])
def test_noalloc_step_matches_rt_step_on_two_calls(case):
    if case == "tiled_fp32":
        big, small, prec = (W.make_problem("c2", scale=(16, 12, 10)),
                            W.make_problem("c2", scale=(8, 8, 6)), rt.RT_F32)
    elif case == "general_fp64":
        big, small, prec = (W.make_problem("c3", scale=(16, 12, 8)),
                            W.make_problem("c3", scale=(8, 6, 4)), rt.RT_F64)
    elif case == "two_stage_fp32":
        big, small, prec = (W.make_problem("c2", scale=(16, 12, 10)),
                            W.make_problem("c2", scale=(8, 8, 6)), rt.RT_F32)
        big.integrator = small.integrator = 2
    else:
        big, small, prec = (W.make_problem("c3", scale=(16, 12, 8)),
                            W.make_problem("c3", scale=(8, 6, 4)), rt.RT_F32)
    for prob in (big, small):              # the second call has the smaller input
        g = rt.Grid(prob, prec, 0)
        dt = g.max_dt(prob.cfl)
        g.close()
        print("noalloc case=%s n=%s nang=%d" % (case, prob.n, prob.nang), flush=True)
        ref = _one_step(prob, prec, False, dt)
        got = _one_step(prob, prec, True, dt)
        assert got[6] == ref[6]
        for a, b in zip(got[:4], ref[:4]):
            assert torch.equal(a, b)
        assert got[4] == ref[4] and got[5] == ref[5]


def test_noalloc_rejects_a_grid_beyond_the_scratch():
    # the general kernel writes one partial per 16 cells: 14.2 M cells need
    # more than the 16 MiB scratch
    n = (242, 242, 242)
    p = W.make_custom("minkowski_cart", n, [(0.0, 1.0)] * 3, 1,
                      [(W.BC_PERIODIC, W.BC_PERIODIC)] * 3)
    p.kernel = 1
    dev = torch.device("cuda", 0)
    g = rt.Grid(p, rt.RT_F32, 0)
    assert g.path == 0
    I = torch.empty((n[2], n[1], n[0], p.nang), dtype=torch.float32, device=dev)
    out = torch.empty_like(I)
    T, rho, ka, ks = (torch.empty((n[2], n[1], n[0]), dtype=torch.float64, device=dev)
                      for _ in range(4))
    u = torch.empty((n[2], n[1], n[0], 3), dtype=torch.float64, device=dev)
    with pytest.raises(rt.RtError, match="static scratch"):
        g.step(I, out, T, rho, u, ka, ks, 1e-3, noalloc=True)
    g.close()
