// Hand-over of the coupling's four-momentum to a gamma-law gas (paper
// Sec. 2.5, last paragraph: the change of the radiation's R^0_alpha leaves
// the gas's T^0_alpha).  One thread per cell, FP64.
//
// In the normal-observer tetrad frame the gas row is E = w u0^2 - p,
// S^a = w u0 u^a (w = rho + Gamma p/(Gamma-1)); the coordinate change dT0
// maps onto it through the per-geometry-cell table gas_map.  The new
// pressure solves
//   r(p) = D gamma + (Gamma/(Gamma-1) gamma^2 - 1) p - E = 0,
//   gamma^2 = X^2 / (X^2 - |S|^2), X = E + p, D = rho u0 (held),
// which is strictly increasing in p for a physical state (r(0) < 0), by
// Newton steps kept inside a shrinking bracket.
#include <hip/hip_runtime.h>

#include "k_transport.h"

namespace rt {
namespace {

constexpr int kGasBlock = 256;
constexpr int kGasMaxIter = 100;

__global__ __launch_bounds__(kGasBlock) void k_gas_update(DevGrid G, const double *__restrict__ dT0,
                                                          const double *Tpre,
                                                          double *__restrict__ rho,
                                                          double *__restrict__ uvec,
                                                          double *T,
                                                          int32_t *__restrict__ status) {
    const long long ncell = (long long)G.n0 * G.n1 * G.n2;
    const long long c = (long long)blockIdx.x * kGasBlock + threadIdx.x;
    if (c >= ncell) return;
    const Cell x = make_cell(G, c);
    const double r0 = rho[c], T0 = Tpre[c];
    const double u1 = uvec[3 * c], u2 = uvec[3 * c + 1], u3 = uvec[3 * c + 2];
    const double u0 = sqrt(1.0 + u1 * u1 + u2 * u2 + u3 * u3);
    const double hf = G.gamma / (G.gamma - 1.0);
    const double p0 = r0 * G.kb * T0;
    const double w = r0 + hf * p0;
    const double *M = G.gas_map + 16 * x.gc;
    const double d0 = dT0[4 * c], d1 = dT0[4 * c + 1], d2 = dT0[4 * c + 2], d3 = dT0[4 * c + 3];
    double row[4] = {w * u0 * u0 - p0, w * u0 * u1, w * u0 * u2, w * u0 * u3};
#pragma unroll
    for (int b = 0; b < 4; ++b)
        row[b] += M[4 * b] * d0 + M[4 * b + 1] * d1 + M[4 * b + 2] * d2 + M[4 * b + 3] * d3;
    const double E = row[0];
    const double S2 = row[1] * row[1] + row[2] * row[2] + row[3] * row[3];
    const double D = r0 * u0;
    // r(p) and r'(p)
    auto resid = [&](double p, double &dr) {
        const double X = E + p;
        const double den = X * X - S2;
        const double g2 = X * X / den;
        const double g = sqrt(g2);
        const double dg2 = -2.0 * X * S2 / (den * den);
        dr = D * dg2 / (2.0 * g) + hf * (g2 + p * dg2) - 1.0;
        return D * g + (hf * g2 - 1.0) * p - E;
    };
    double dr = 0.0;
    int ok = E > 0.0 && E * E > S2 && resid(0.0, dr) < 0.0;
    double p = 0.0;
    if (ok) {
        double lo = 0.0, hi = E;
        int k = 0;
        while (resid(hi, dr) <= 0.0 && k < 64) {
            lo = hi;
            hi *= 2.0;
            ++k;
        }
        ok = resid(hi, dr) > 0.0;
        p = (p0 > lo && p0 < hi) ? p0 : 0.5 * (lo + hi);
        for (int it = 0; ok && it < kGasMaxIter; ++it) {
            const double rv = resid(p, dr);
            if (rv == 0.0) break;
            if (rv < 0.0) lo = p;
            else hi = p;
            double pn = p - rv / dr;
            if (!(pn > lo && pn < hi)) pn = 0.5 * (lo + hi);
            const bool done = fabs(pn - p) <= 1e-15 * pn || pn == lo || pn == hi;
            p = pn;
            if (done) break;
        }
    }
    if (status) status[c] = ok ? 0 : 1;
    if (!ok) return;
    const double X = E + p;
    const double g = X / sqrt(X * X - S2);
    const double rn = D / g;
    rho[c] = rn;
    uvec[3 * c] = g * row[1] / X;
    uvec[3 * c + 1] = g * row[2] / X;
    uvec[3 * c + 2] = g * row[3] / X;
    T[c] = p / (rn * G.kb);
}

}  // namespace

int launch_gas_update(rt_grid *g, hipStream_t s, const double *dT0, const double *Tpre,
                      double *rho, double *u, double *T, int32_t *status) {
    const long long ncell = (long long)g->dg.n0 * g->dg.n1 * g->dg.n2;
    const int nblk = (int)((ncell + kGasBlock - 1) / kGasBlock);
    if (nblk == 0) return RT_OK;
    hipLaunchKernelGGL(k_gas_update, dim3(nblk), dim3(kGasBlock), 0, s, g->dg, dT0, Tpre, rho, u,
                       T, status);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_EDEVICE;
}

}  // namespace rt
