"""Pins of the oracle's two-stage integrator and optical-depth-aware flux.

R1  two-stage (Heun) integrator, vacuum donor-cell transport: every Fourier
    mode of every direction is multiplied per step by 1 + z + z^2/2, the
    stability polynomial of Heun's method, z = (forward-Euler symbol) - 1;
R2  two-stage integrator, static equilibration: total energy (radiation +
    gas) is conserved to round-off every step and T relaxes to the T_eq of
    the closed-form energy balance (the same fixed point as one stage);
R3  optical-depth-aware flux: with a spatially uniform velocity the factor
    (1 - g_up + g) is exactly 1, so the step equals free streaming bit for
    bit whatever the opacities (Sec. 2, flux calculation);
R4  the optical-depth-aware flux keeps the flux form: in a periodic box the
    transport moves no energy, sum_c dV q (I* - I) = 0 per direction.
R5  the factor departs from 1 as tau^2 at small optical depth and saturates
    (f = 1) at large optical depth;
R6  two stages + tau flux, static diffusion (Sec. 3): the energy pulse
    converges to the diffusion solution of the paper as resolution grows.
The size of the factor's effect under velocity gradients rests on a reading
of the paper (g = (g_L + g_R)/2) and is parity unpinned.
"""
import json
import math
import os

import numpy as np
import torch

from oracle import step as O
from paper_2302_04283_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
EQ = GOLD["static_equilibration"]
T_EQ = 1.214799340993827


def _cart(n, nlev, recon=W.RECON_PLM, bc=W.BC_PERIODIC):
    return W.make_custom("minkowski_cart", n, [(0.0, 1.0)] * 3, nlev,
                         [(bc, bc)] * 3, recon=recon)


def _heun_fourier(I0, nhat, nu_dt, steps):
    out = np.empty_like(I0)
    n2, n1, n0, N = I0.shape
    k = [2 * np.pi * np.fft.fftfreq(m) for m in (n0, n1, n2)]
    K0 = k[0][None, None, :]
    K1 = k[1][None, :, None]
    K2 = k[2][:, None, None]
    for a in range(N):
        nu = np.abs(nhat[a]) * nu_dt
        s = np.sign(nhat[a])
        z = (-nu.sum() + nu[0] * np.exp(-1j * s[0] * K0)
             + nu[1] * np.exp(-1j * s[1] * K1) + nu[2] * np.exp(-1j * s[2] * K2))
        G = 1.0 + z + 0.5 * z * z
        out[..., a] = np.real(np.fft.ifftn(np.fft.fftn(I0[..., a]) * G ** steps))
    return out


def test_r1_two_stage_donor_cell_fourier():
    p = _cart((8, 6, 5), 2, recon=W.RECON_DC)
    p.integrator = 2
    S = O.setup(p)
    rng = np.random.default_rng(5)
    I0 = rng.random((5, 6, 8, p.nang))
    dt = 0.05
    I, T, _, _ = O.run(p, S, I0, p.T, dt, 7)
    dx = np.array([1 / 8, 1 / 6, 1 / 5])
    exp = _heun_fourier(I0, S.ang.nhat, dt / dx, 7)
    assert np.abs(I.numpy() - exp).max() <= 1e-13
    # and one stage is not the same thing
    p1 = _cart((8, 6, 5), 2, recon=W.RECON_DC)
    I1, _, _, _ = O.run(p1, O.setup(p1), I0, p1.T, dt, 7)
    assert np.abs(I1.numpy() - exp).max() > 1e-6


def test_r2_two_stage_equilibration_conserves_energy():
    p = _cart((4, 4, 4), 2)
    p.integrator = 2
    p.gamma_gas = EQ["gamma"]
    p.rho[:] = EQ["rho"]
    p.T[:] = EQ["p_gas0"] / EQ["rho"]
    p.kappa_a[:] = EQ["alpha_a"] / EQ["rho"]
    S = O.setup(p)
    rho, u, ka, ks = O.fluid_tensors(p)
    I = torch.full((4, 4, 4, p.nang), 1.0 / (4 * math.pi), dtype=torch.float64)
    T = torch.full((4, 4, 4), 2.0, dtype=torch.float64)
    cv = 1.0 / (EQ["gamma"] - 1.0)
    E0 = float((I[0, 0, 0] * S.domega).sum()) + EQ["rho"] * cv * 2.0
    for _ in range(200):
        I, T, _, _ = O.step(I, T, S, rho, u, ka, ks, 1.0)
        E = float((I[0, 0, 0] * S.domega).sum()) + EQ["rho"] * cv * float(T[0, 0, 0])
        assert abs(E - E0) <= 1e-14 * E0
    assert abs(float(T[0, 0, 0]) - T_EQ) <= 1e-12
    assert float((T - T[0, 0, 0]).abs().max()) == 0.0


def test_r3_tau_flux_uniform_flow_is_free_streaming():
    p = W.make_problem("c2", scale=(8, 6, 6))
    p.u_tet[:] = np.array([0.3, -0.2, 0.1])          # one velocity everywhere
    p.beam_mask = None
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    I0 = p.initial_intensity()
    Ia, Ta, da, Ja = O.run(p, S, I0, p.T, dt, 3)
    p.tau_coeff = 5.0                                  # opacities vary cell to cell
    Ib, Tb, db, Jb = O.run(p, O.setup(p), I0, p.T, dt, 3)
    assert torch.equal(Ia, Ib) and torch.equal(Ta, Tb) and float(Ja) == float(Jb)


def test_r4_tau_flux_keeps_flux_form():
    p = W.make_problem("c2", scale=(8, 6, 6))          # random velocities and opacities
    p.tau_coeff = 5.0
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    fl = O.fluid_tensors(p)
    I = torch.as_tensor(p.initial_intensity())
    Is, _ = O.transport(I, S, dt, None, fl)
    Is0, _ = O.transport(I, S, dt, None, None)
    assert float((Is - Is0).abs().max()) > 1e-8 * float(I.abs().max())   # the factor acts
    moved = ((S.q * (Is - I)) * S.vol[..., None]).sum((0, 1, 2))
    scale = ((S.q * I).abs() * S.vol[..., None]).sum((0, 1, 2))
    assert float((moved / scale).abs().max()) <= 1e-14


def test_r5_tau_flux_onset_is_quadratic_and_saturates():
    """f = -expm1(-tau^2): the factor's departure from 1 grows as tau^2 for
    small optical depth (so as C_tau^2 at fixed fields) and stops growing
    once f reaches 1 (tau^2 beyond double precision's reach of exp)."""
    p = W.make_problem("c2", scale=(8, 6, 6))
    S = O.setup(p)
    dt = O.max_dt(S, 0.3)
    fl = O.fluid_tensors(p)
    I = torch.as_tensor(p.initial_intensity())
    Is0, _ = O.transport(I, S, dt, None, None)

    def dev(c):
        p.tau_coeff = c
        return O.transport(I, S, dt, None, fl)[0] - Is0

    d1, d2 = dev(1e-3), dev(2e-3)
    assert float(d1.abs().max()) > 0.0
    assert float((d2 - 4.0 * d1).abs().max()) <= 1e-4 * float(d2.abs().max())
    big1, big2 = dev(1e5), dev(1e6)
    assert torch.isfinite(big1).all() and torch.equal(big1, big2)
    assert float(big1.abs().max()) > float(d2.abs().max())


def _diffusion_error(N, alpha_s=1000.0, sigma=0.1, A_end=0.8):
    """Static diffusion (Sec. 3): a Gaussian energy pulse in a purely
    scattering medium at rest; returns the max error of E(x) against the
    diffusion solution E = A exp(-A^2 x^2 / 2 sigma^2), sigma^2 -> sigma^2 / A^2
    with D = 1/(3 alpha_s), and the relative change of the total energy."""
    dx = 2.0 / N
    p = W.make_custom("minkowski_cart", (N, 2, 2), [(-1.0, 1.0), (0.0, 2 * dx), (0.0, 2 * dx)], 1,
                      [(W.BC_PERIODIC, W.BC_PERIODIC)] * 3)
    p.kappa_s[:] = alpha_s
    p.integrator, p.tau_coeff = 2, 5.0
    S = O.setup(p)
    t_end = (1.0 / A_end ** 2 - 1.0) * 1.5 * alpha_s * sigma ** 2
    nsteps = int(math.ceil(t_end / O.max_dt(S, 0.3)))
    x = -1.0 + dx * (np.arange(N) + 0.5)
    E0 = np.exp(-x ** 2 / (2 * sigma ** 2))
    I0 = np.broadcast_to((E0 / (4 * np.pi))[None, None, :, None], (2, 2, N, p.nang)).copy()
    I, _, _, _ = O.run(p, S, I0, p.T, t_end / nsteps, nsteps)
    E = (I * S.domega).sum(-1)[0, 0].numpy()
    Ex = A_end * np.exp(-A_end ** 2 * x ** 2 / (2 * sigma ** 2))
    return float(np.abs(E - Ex).max()), abs(E.sum() / E0.sum() - 1.0)


def test_r6_two_stage_static_diffusion_converges_to_the_gaussian():
    """Two stages with the tau flux in the optically thick limit (12
    directions, per-cell scattering depth 15-60): the pulse spreads at the
    physical rate as resolution grows, the error falling at close to second
    order once the cells resolve the pulse; energy is conserved throughout."""
    errs = []
    for N in (32, 64, 128):
        e, de = _diffusion_error(N)
        assert de <= 1e-11          # round-off over up to 1800 stages
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[2] >= 3.0
    assert errs[2] <= 0.07
