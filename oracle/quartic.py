"""Root of the coupling quartic  B4 T^4 + B1 T + B0 = 0  (paper Sec. 2.5).

With B4 >= 0, B1 > 0 and B0 < 0 the polynomial is increasing on T >= 0 and has
exactly one positive root, bracketed by [0, T_hi] with
T_hi = min(-B0/B1, (-B0/B4)^(1/4)) since each single term alone already
overshoots zero there.  The oracle bisects that bracket (200 halvings, far
more than the 53 bits of a double need) and finishes with one Newton step.

Edge cases (the paper is silent): B4 = 0 gives the linear root -B0/B1;
B0 >= 0 or a non-finite coefficient has no positive root, in which case the
result is 1e-12 and the cell is counted.  A root that over- or underflows
the double range (outside (0, 1e300): coefficients near its ends) is no
usable temperature either and takes the same floor, counted.

The backward pass uses the implicit-function theorem:
dT/dB_k = -T^k / (4 B4 T^3 + B1), k = 4, 1, 0.

Pins: 400 random coefficient sets with B4/B1 over 24 decades (and B4 = 0)
against 50-digit mpmath roots to 4 ulp, and the no-root counting, in
tests/test_oracle_step.py (P10); the static-equilibration closed form T_eq
(P7) exercises it inside the coupling.
"""
from __future__ import annotations

import torch

NO_ROOT_T = 1e-12


def _solve(B4, B1, B0):
    ok = torch.isfinite(B4) & torch.isfinite(B1) & torch.isfinite(B0) & (B0 < 0) & (B1 > 0)
    lin = -B0 / torch.where(B1 > 0, B1, torch.ones_like(B1))
    quart = torch.where(B4 > 0, (-B0 / torch.where(B4 > 0, B4, torch.ones_like(B4))) ** 0.25,
                        torch.full_like(B4, float("inf")))
    hi = torch.minimum(lin, quart)
    lo = torch.zeros_like(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        p = B4 * mid ** 4 + B1 * mid + B0
        pos = p > 0
        hi = torch.where(pos, mid, hi)
        lo = torch.where(pos, lo, mid)
    T = 0.5 * (lo + hi)
    p = B4 * T ** 4 + B1 * T + B0
    dp = 4.0 * B4 * T ** 3 + B1
    T = T - p / dp
    T = torch.where(B4 > 0, T, lin)
    ok = ok & (T > 0) & (T < 1e300)
    nbad = int((~ok).sum())
    T = torch.where(ok, T, torch.full_like(T, NO_ROOT_T))
    return T, nbad


class _QuarticRoot(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B4, B1, B0):
        T, nbad = _solve(B4.detach(), B1.detach(), B0.detach())
        ctx.save_for_backward(T, B4, B1)
        ctx.nbad = nbad
        return T

    @staticmethod
    def backward(ctx, gT):
        T, B4, B1 = ctx.saved_tensors
        den = 4.0 * B4 * T ** 3 + B1
        s = -gT / den
        return s * T ** 4, s * T, s


def quartic_root(B4, B1, B0):
    """Positive root per element; differentiable via the implicit function theorem."""
    return _QuarticRoot.apply(B4, B1, B0)


def quartic_root_count(B4, B1, B0):
    """(root, number of elements with no positive root)."""
    return _solve(B4, B1, B0)
