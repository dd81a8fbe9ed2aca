"""The hand-written adjoint (rt_step_adjoint through RadTransport) against the
oracle's reference gradient and against central finite differences.

Tolerances: FP64 adjoint vs the oracle's autograd gradient 1e-10 in max-norm
relative to max|g|; FP32 adjoint 1e-4; FP64 adjoint vs central differences
(h = 1e-6 relative) 1e-5 relative on cells with a non-negligible gradient,
plus the cancellation floor of a central difference, 4e-15 |J| / h (the two
perturbed runs each carry ~1e-15 |J| of rounding in their FP64 sums).
"""
import numpy as np
import pytest
import torch

from oracle import gradient as GR
from oracle import step as O
from paper_2302_04283_amd import rt
from paper_2302_04283_amd import workloads as W
from paper_2302_04283_amd.autograd import luminosity_and_gradients

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(DEV)


def _gpu_grads(p, prec, steps, dt, K, I0=None, T0=None):
    g = rt.Grid(p, prec)
    I0 = p.initial_intensity() if I0 is None else I0
    T0 = p.T if T0 is None else T0
    J, gI, gT, gka, gks = luminosity_and_gradients(
        g, _t(I0).to(g.real_dtype()), _t(T0), _t(p.kappa_a), _t(p.kappa_s), _t(p.rho),
        _t(p.u_tet), dt, steps, K)
    out = {"J": float(J), "I0": gI.double().cpu().numpy(), "T0": gT.cpu().numpy(),
           "kappa_a": gka.cpu().numpy(), "kappa_s": gks.cpu().numpy()}
    g.close()
    return out


def _max_rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("cfg,scale,steps,K", [("c4", (12, 8, 6), 6, 4), ("c3", (10, 8, 4), 4, 2),
                                               ("c2", (8, 8, 8), 5, 2), ("c5", (6, 4, 4), 3, 2)])
@pytest.mark.parametrize("prec", [rt.RT_F64, rt.RT_F32])
def test_adjoint_matches_reference_gradient(cfg, scale, steps, K, prec):
    p = W.make_problem(cfg, scale=scale)
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    ref = GR.reference_gradient(p, p.initial_intensity(), p.T, dt, steps)
    got = _gpu_grads(p, prec, steps, dt, K)
    tol = 1e-10 if prec == rt.RT_F64 else 1e-4
    errs = {k: _max_rel(got[k], ref[k]) for k in ("kappa_a", "kappa_s", "T0", "I0")}
    eJ = abs(got["J"] - ref["J"]) / abs(ref["J"])
    print("[adjoint] %s %s %s steps=%d K=%d e_J=%.2e %s" % (
        cfg, scale, "fp64" if prec == rt.RT_F64 else "fp32", steps, K, eJ,
        " ".join("e_%s=%.2e" % kv for kv in errs.items())), flush=True)
    for k, e in errs.items():
        assert e <= tol, (k, e)


def test_adjoint_checkpoint_interval_does_not_change_gradients():
    p = W.make_problem("c4", scale=(12, 8, 6))
    dt = O.max_dt(O.setup(p), 0.3)
    a = _gpu_grads(p, rt.RT_F64, 7, dt, 1)
    b = _gpu_grads(p, rt.RT_F64, 7, dt, 7)
    c = _gpu_grads(p, rt.RT_F64, 7, dt, 3)
    for k in ("kappa_a", "T0", "I0"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k])


def test_adjoint_full_c4_central_differences():
    """64x32x64, 92 directions, 50 steps, checkpoint every 10 steps (FP64):
    16 kappa_a cells and 16 T0 cells among those with |g| >= 1e-3 max|g|
    whose central-difference signal |g| h is resolvable (>= 1e-9 |J|), plus,
    as controls, the 4 cells with the smallest |g| (their central difference
    must be negligible against max|g|)."""
    p = W.make_problem("c4")
    dt = O.max_dt(O.setup(p), p.cfl)
    steps, K = p.nsteps, 10
    got = _gpu_grads(p, rt.RT_F64, steps, dt, K)
    g = rt.Grid(p, rt.RT_F64)
    I0 = _t(p.initial_intensity())
    rho, u, ks = _t(p.rho), _t(p.u_tet), _t(p.kappa_s)

    def J_of(ka, T0):
        I = I0.clone()
        Ib = torch.empty_like(I)
        T = T0.clone()
        lum = torch.zeros(1, dtype=torch.float64, device=DEV)
        for _ in range(steps):
            g.step(I, Ib, T, rho, u, ka, ks, dt, None, lum)
            I, Ib = Ib, I
        return float(lum[0])

    J0 = got["J"]
    rng = np.random.default_rng(4)
    worst = 0.0
    for key in ("kappa_a", "T0"):
        G = got[key]
        hh = 1e-6 * (p.kappa_a if key == "kappa_a" else p.T)
        # cells with a non-negligible gradient, largest finite-difference signal first
        signal = (np.abs(G) * hh / abs(J0)).ravel()
        cand = np.flatnonzero(np.abs(G).ravel() >= 1e-3 * np.abs(G).max())
        cand = cand[np.argsort(-signal[cand])]
        pick = cand[:16]
        assert pick.size >= 8 and signal[pick[7]] >= 1e-13, (key, pick.size, signal[pick[:8]])
        small = np.argsort(np.abs(G).ravel())[:4]
        gmax = np.abs(G).max()
        for flat in np.concatenate([pick, small]):
            c = np.unravel_index(flat, G.shape)
            base_ka = _t(p.kappa_a)
            base_T = _t(p.T)
            if key == "kappa_a":
                h = 1e-6 * p.kappa_a[c]
                kp, km = base_ka.clone(), base_ka.clone()
                kp[c] += h
                km[c] -= h
                fd = (J_of(kp, base_T) - J_of(km, base_T)) / (2 * h)
            else:
                h = 1e-6 * p.T[c]
                tp, tm = base_T.clone(), base_T.clone()
                tp[c] += h
                tm[c] -= h
                fd = (J_of(base_ka, tp) - J_of(base_ka, tm)) / (2 * h)
            floor = 4e-15 * abs(J0) / h
            if flat in small:
                assert abs(fd - G[c]) <= 1e-6 * gmax + floor, (key, c, G[c], fd)
            else:
                e = abs(G[c] - fd) / abs(G[c])
                worst = max(worst, e)
                assert abs(G[c] - fd) <= 1e-5 * abs(G[c]) + floor, (key, c, G[c], fd, floor)
    print("[adjoint] c4 full 64x32x64x92 50 steps K=10: worst FD rel err %.2e "
          "(central differences, h = 1e-6 relative)" % worst, flush=True)
    g.close()


# ------------------------------------------------------- stored I*, tiled adjoint
@pytest.mark.parametrize("prec", [rt.RT_F64, rt.RT_F32])
@pytest.mark.parametrize("case", ["fast", "general"])
def test_step_I_star_output_matches_oracle_transport(case, prec):
    """rt_step's optional I* output is the oracle's transport result (before
    the coupling), masked directions zero."""
    if case == "fast":
        p = W.make_problem("c2", scale=(8, 12, 5), nlev=3)
    else:
        p = W.make_problem("c4", scale=(12, 8, 6))
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    I0 = p.initial_intensity()
    ref, _ = O.transport(torch.as_tensor(I0), S, dt)
    ref = ref.numpy()
    g = rt.Grid(p, prec)
    assert g.fast_path == (case == "fast")
    rd = g.real_dtype()
    I = _t(I0).to(rd)
    Ib = torch.empty_like(I)
    Is = torch.full_like(I, float("nan"))
    g.step(I, Ib, _t(p.T), _t(p.rho), _t(p.u_tet), _t(p.kappa_a), _t(p.kappa_s), dt,
           I_star=Is)
    got = Is.double().cpu().numpy()
    g.close()
    scale = np.abs(ref) + 1e-3 * np.abs(ref).max()
    e = float(np.max(np.abs(got - ref) / scale))
    print("[adjoint] I* output %s %s e=%.2e" % (case, "fp64" if prec == 0 else "fp32", e),
          flush=True)
    assert np.isfinite(got).all()
    assert e <= (1e-12 if prec == rt.RT_F64 else 1e-5)


def _tiled_problem(bc, lum_axis, lum_side, shape=(8, 8, 7), nlev=3, seed=5):
    p = W.make_custom("minkowski_cart", shape, [(0.0, 1.0)] * 3, nlev, bc)
    rng = np.random.default_rng(seed)
    shp = p.T.shape
    p.T[:] = 0.5 + rng.random(shp)
    p.kappa_a[:] = 4.0 * rng.random(shp)
    p.kappa_s[:] = 4.0 * rng.random(shp)
    p.rho[:] = 0.5 + rng.random(shp)
    p.u_tet[:] = 0.3 * (rng.random(shp + (3,)) - 0.5)
    p.lum_axis, p.lum_side = lum_axis, lum_side
    return p


PER = [(0, 0)] * 3
OUT = [(1, 1)] * 3


BOUNDARY_CASES = [
    (PER, 0, 1), (PER, 1, 0), (PER, 2, 1), (PER, 2, 0),
    (OUT, 0, 0), (OUT, 1, 1), (OUT, 2, 0), (OUT, 2, 1),
    ([(0, 0), (1, 1), (0, 0)], 1, 0)]


def _bc_tag(bc):
    return "per" if bc == PER else ("out" if bc == OUT else "mixed")


@pytest.mark.parametrize("bc,lum_axis,lum_side", BOUNDARY_CASES)
def test_tiled_adjoint_boundaries_and_luminosity_faces(bc, lum_axis, lum_side):
    """The tiled transport adjoint (uniform geometry, FP64) against the
    oracle's reference gradient for every luminosity face and both boundary
    kinds."""
    p = _tiled_problem(bc, lum_axis, lum_side)
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    steps = 4
    I0 = np.abs(p.initial_intensity()) + 0.1
    ref = GR.reference_gradient(p, I0, p.T, dt, steps)
    g = rt.Grid(p, rt.RT_F64)
    assert g.fast_path
    g.close()
    got = _gpu_grads(p, rt.RT_F64, steps, dt, 2, I0=I0)
    errs = {k: _max_rel(got[k], ref[k]) for k in ("kappa_a", "kappa_s", "T0", "I0")}
    print("[adjoint] tiled bc=%s lum=(%d,%d) fp64 %s" % (
        _bc_tag(bc), lum_axis, lum_side, " ".join("e_%s=%.2e" % kv for kv in errs.items())),
        flush=True)
    for k, e in errs.items():
        assert e <= 1e-10, (k, e)


def _manual_adjoint(g, states, rho, u, ka, ks, dt):
    I = states[0][0]
    lamI, lamT = torch.zeros_like(I), torch.zeros_like(states[0][1])
    work = torch.empty_like(I)
    gka, gks = torch.zeros_like(lamT), torch.zeros_like(lamT)
    for Is, Ts in reversed(states):
        g.step_adjoint(Is, Ts, rho, u, ka, ks, dt, lamI, lamT, lamI, lamT, work, gka, gks)
    return {"I0": lamI.double().cpu().numpy(), "T0": lamT.cpu().numpy(),
            "kappa_a": gka.cpu().numpy(), "kappa_s": gks.cpu().numpy()}


@pytest.mark.parametrize("bc,lum_axis,lum_side", BOUNDARY_CASES)
def test_tiled_adjoint_fp32_arithmetic(bc, lum_axis, lum_side):
    """FP32 adjoint = exact derivative of the FP32 step.  Against the FP64
    reference it can differ by far more than rounding wherever the FP32
    trajectory takes the other branch of a van Leer limiter (the gradient of
    a limited scheme jumps there; on the periodic, luminosity-face-0 case of
    this set one direction flips and the FP32 gradient is 1e-2 off in
    max-norm).  So the FP32 adjoint arithmetic is checked against the FP64
    library adjoint evaluated on the same FP32 trajectory (1e-5), and the
    FP32 trajectory against the oracle (forward parity)."""
    p = _tiled_problem(bc, lum_axis, lum_side)
    dt = O.max_dt(O.setup(p), 0.3)
    I0 = np.abs(p.initial_intensity()) + 0.1
    g32, g64 = rt.Grid(p, rt.RT_F32), rt.Grid(p, rt.RT_F64)
    assert g32.fast_path and g64.fast_path
    rho, u, ka, ks = _t(p.rho), _t(p.u_tet), _t(p.kappa_a), _t(p.kappa_s)
    I, T = _t(I0).float(), _t(p.T)
    states = []
    for _ in range(4):
        Ib = torch.empty_like(I)
        states.append((I.clone(), T.clone()))
        g32.step(I, Ib, T, rho, u, ka, ks, dt)
        I = Ib
    a = _manual_adjoint(g32, states, rho, u, ka, ks, dt)
    b = _manual_adjoint(g64, [(Is.double(), Ts) for Is, Ts in states], rho, u, ka, ks, dt)
    g32.close()
    g64.close()
    errs = {k: _max_rel(a[k], b[k]) for k in ("kappa_a", "kappa_s", "T0", "I0")}
    print("[adjoint] tiled fp32 arithmetic bc=%s lum=(%d,%d) %s" % (
        _bc_tag(bc), lum_axis, lum_side, " ".join("e_%s=%.2e" % kv for kv in errs.items())),
        flush=True)
    for k, e in errs.items():
        assert e <= 1e-5, (k, e)


@pytest.mark.parametrize("nlev,shape,seglen", [(4, (8, 4, 7), "3"), (2, (4, 8, 5), "2"),
                                               (1, (4, 4, 3), "1"), (3, (4, 4, 6), "4")])
def test_tiled_adjoint_matches_general_adjoint(nlev, shape, seglen):
    """Tiled and general adjoint on the same inputs (FP64): direction chunks
    (162 directions span two chunks of 96, 92 one padded chunk), ragged
    segments along axis 2."""
    p = W.make_problem("c2", scale=shape, nlev=nlev)
    dt = O.max_dt(O.setup(p), 0.3)
    p.seglen = int(seglen)
    g = rt.Grid(p, rt.RT_F64)
    assert g.fast_path
    g.close()
    a = _gpu_grads(p, rt.RT_F64, 3, dt, 3)
    p.kernel = 1
    b = _gpu_grads(p, rt.RT_F64, 3, dt, 3)
    errs = {k: _max_rel(a[k], b[k]) for k in ("kappa_a", "kappa_s", "T0", "I0")}
    print("[adjoint] tiled vs general lev%d %s seglen %s %s" % (
        nlev, shape, seglen, " ".join("e_%s=%.2e" % kv for kv in errs.items())), flush=True)
    for k, e in errs.items():
        assert e <= 1e-12, (k, e)


def test_adjoint_with_and_without_stored_I_star():
    """rt_step_adjoint given I* equals the adjoint that recomputes it."""
    p = W.make_problem("c4", scale=(12, 8, 6))
    dt = O.max_dt(O.setup(p), 0.3)
    g = rt.Grid(p, rt.RT_F64)
    I0 = _t(p.initial_intensity())
    T0, rho, u, ka, ks = _t(p.T), _t(p.rho), _t(p.u_tet), _t(p.kappa_a), _t(p.kappa_s)
    I1, Is = torch.empty_like(I0), torch.empty_like(I0)
    T1 = T0.clone()
    g.step(I0, I1, T1, rho, u, ka, ks, dt, I_star=Is)
    rng = np.random.default_rng(11)
    lamI1 = _t(rng.standard_normal(tuple(I0.shape)))
    lamT1 = _t(rng.standard_normal(tuple(T0.shape)))
    outs = []
    for star in (None, Is):
        lI, lT, work = torch.empty_like(I0), torch.empty_like(T0), torch.empty_like(I0)
        gka, gks = torch.zeros_like(T0), torch.zeros_like(T0)
        g.step_adjoint(I0, T0, rho, u, ka, ks, dt, lamI1, lamT1, lI, lT, work, gka, gks,
                       lum_weight=0.7, I_star=star)
        outs.append([x.cpu().numpy() for x in (lI, lT, gka, gks)])
    g.close()
    for x, y in zip(*outs):
        assert _max_rel(x, y) <= 1e-13
