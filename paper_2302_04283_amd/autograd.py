"""Differentiable driver: N radiation steps as one torch.autograd.Function.

J = sum over steps of dt * l(I_s), the energy leaving through the grid's
luminosity face.  The forward pass runs the HIP step and keeps a checkpoint of
(I, T) every K steps; the backward pass walks the segments newest first,
recomputes the K states of a segment from its checkpoint, and applies the
hand-written adjoint step (rt_step_adjoint) in reverse.  Memory is
ceil(N/K) checkpoints + K segment states and K transport results (I*) +
three adjoint buffers.

Gradients are returned for the initial intensities, the initial gas
temperature and the per-cell absorption and scattering opacities.
"""
from __future__ import annotations

import torch


class RadTransport(torch.autograd.Function):
    @staticmethod
    def forward(ctx, I0, T0, kappa_a, kappa_s, grid, rho, u, dt, nsteps, K):
        K = max(1, int(K))
        I = I0.detach().clone()
        Ib = torch.empty_like(I)
        T = T0.detach().clone()
        ka = kappa_a.detach().contiguous()
        ks = kappa_s.detach().contiguous()
        lum = torch.zeros(1, dtype=torch.float64, device=I.device)
        ckpts = []
        for s in range(nsteps):
            if s % K == 0:
                ckpts.append((I.clone(), T.clone()))
            grid.step(I, Ib, T, rho, u, ka, ks, dt, None, lum)
            I, Ib = Ib, I
        ctx.grid, ctx.rho, ctx.u, ctx.dt, ctx.nsteps, ctx.K = grid, rho, u, dt, nsteps, K
        ctx.ckpts = ckpts
        ctx.ka, ctx.ks = ka, ks
        return lum[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        g, rho, u, dt, K = ctx.grid, ctx.rho, ctx.u, ctx.dt, ctx.K
        ka, ks = ctx.ka, ctx.ks
        w = float(gJ)
        I0, T0 = ctx.ckpts[0]
        lamI = torch.zeros_like(I0)
        lamT = torch.zeros_like(T0)
        work = torch.empty_like(I0)
        gka = torch.zeros_like(ka)
        gks = torch.zeros_like(ks)
        # segment buffers: the K states, and I* of each step (the transport
        # result the forward step hands to the coupling), so the adjoint
        # step does not recompute the transport
        nK = min(K, ctx.nsteps)
        Ibuf = [torch.empty_like(I0) for _ in range(nK + 1)]
        Sbuf = [torch.empty_like(I0) for _ in range(nK)]
        Tbuf = [torch.empty_like(T0) for _ in range(nK)]
        nseg = len(ctx.ckpts)
        for seg in reversed(range(nseg)):
            s0 = seg * K
            s1 = min(ctx.nsteps, s0 + K)
            Ibuf[0].copy_(ctx.ckpts[seg][0])
            T = ctx.ckpts[seg][1].clone()
            for j in range(s1 - s0):
                Tbuf[j].copy_(T)
                g.step(Ibuf[j], Ibuf[j + 1], T, rho, u, ka, ks, dt, I_star=Sbuf[j])
            for j in reversed(range(s1 - s0)):
                g.step_adjoint(Ibuf[j], Tbuf[j], rho, u, ka, ks, dt, lamI, lamT, lamI, lamT, work,
                               gka, gks, lum_weight=w, I_star=Sbuf[j])
        ctx.ckpts = None
        return lamI, lamT, gka, gks, None, None, None, None, None, None


def luminosity_and_gradients(grid, I0, T0, kappa_a, kappa_s, rho, u, dt, nsteps, K):
    """Convenience wrapper: (J, dJ/dI0, dJ/dT0, dJ/dkappa_a, dJ/dkappa_s)."""
    I = I0.detach().clone().requires_grad_(True)
    T = T0.detach().clone().requires_grad_(True)
    ka = kappa_a.detach().clone().requires_grad_(True)
    ks = kappa_s.detach().clone().requires_grad_(True)
    J = RadTransport.apply(I, T, ka, ks, grid, rho, u, dt, nsteps, K)
    J.backward()
    return J.detach(), I.grad, T.grad, ka.grad, ks.grad
