#!/usr/bin/env python3
"""Benchmark of the fused radiation step on one MI355X.

Workload: Minkowski Cartesian 128^3 periodic box, geodesic level 4 (162
directions), random fluid velocities |v| <= 0.5, lognormal absorption and
scattering, collimated beam; FP32 intensities with the FP64 quartic and
bookkeeping.  A step is one pass of the whole hot path: boundary handling,
reconstruction, spatial and angular fluxes, divergence, primitives, the
|n_0| mask, the implicit coupling with its quartic, four-momentum
bookkeeping and the luminosity.  Inputs are resident in HBM before the timed
region starts.

Prints one JSON line: value = cell-angle updates per second (FP32 path),
plus the plain-FP64 rate, the roofline of the step kernel and the CPU
oracle's rate on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CONFIG = "c2"


def _upload_initial(prob, dtype, dev):
    import numpy as np
    import torch
    out = torch.empty((prob.n[2], prob.n[1], prob.n[0], prob.nang), dtype=dtype, device=dev)
    for kr, arr in prob.initial_intensity_slabs(np.float64):
        out[kr[0]:kr[1]] = torch.as_tensor(arr).to(dev, dtype)
    return out


def _kernel_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2302_04283_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2302_04283_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(bytes_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_step_c2.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != _kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def time_path(prob, precision, steps, warmup, dt, dev):
    import torch
    from paper_2302_04283_amd import rt
    g = rt.Grid(prob, precision, dev.index or 0)
    print("[bench] %s path: %s kernel" % ("fp32" if precision == rt.RT_F32 else "fp64",
                                         "tiled" if g.fast_path else "general"),
          file=sys.stderr, flush=True)
    Ia = _upload_initial(prob, g.real_dtype(), dev)
    Ib = torch.empty_like(Ia)
    T = torch.as_tensor(prob.T).to(dev)
    rho, u, ka, ks = (torch.as_tensor(x).to(dev) for x in
                      (prob.rho, prob.u_tet, prob.kappa_a, prob.kappa_s))
    dT0 = torch.zeros(T.shape + (4,), dtype=torch.float64, device=dev)
    lum = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        g.step(Ia, Ib, T, rho, u, ka, ks, dt, dT0, lum)
        Ia, Ib = Ib, Ia
    torch.cuda.synchronize(dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        evs[s][0].record()
        g.step(Ia, Ib, T, rho, u, ka, ks, dt, dT0, lum)
        evs[s][1].record()
        Ia, Ib = Ib, Ia
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) * 1e-3 for a, b in evs]
    st = g.stats()
    g.close()
    del Ia, Ib
    torch.cuda.empty_cache()
    return wall, per, st


def time_gas_update(prob, dev, reps):
    """Average duration of rt_gas_update over the workload's cells (the
    change dT0 is zero, so every call starts from the same gas state)."""
    import torch
    from paper_2302_04283_amd import rt
    g = rt.Grid(prob, rt.RT_F64, dev.index or 0)
    T = torch.as_tensor(prob.T).to(dev)
    rho, u = torch.as_tensor(prob.rho).to(dev), torch.as_tensor(prob.u_tet).to(dev)
    d0 = torch.zeros(T.shape + (4,), dtype=torch.float64, device=dev)
    Tp = T.clone()
    g.gas_update(d0, Tp, rho, u, T)
    torch.cuda.synchronize(dev)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.gas_update(d0, Tp, rho, u, T)
    b.record()
    torch.cuda.synchronize(dev)
    g.close()
    return a.elapsed_time(b) * 1e-3 / reps


def time_fwd_adjoint(prob, precision, steps, ckpt, dt, dev):
    """Forward with a checkpoint every `ckpt` steps plus the hand-written
    adjoint (segment recompute + reverse steps): whole-job wall time."""
    import torch
    from paper_2302_04283_amd import rt
    from paper_2302_04283_amd.autograd import RadTransport
    g = rt.Grid(prob, precision, dev.index or 0)
    I0 = _upload_initial(prob, g.real_dtype(), dev)
    T0 = torch.as_tensor(prob.T).to(dev)
    rho, u, ka, ks = (torch.as_tensor(x).to(dev) for x in
                      (prob.rho, prob.u_tet, prob.kappa_a, prob.kappa_s))

    def run(n):
        kk = ka.clone().requires_grad_(True)
        tt = T0.clone().requires_grad_(True)
        J = RadTransport.apply(I0, tt, kk, ks, g, rho, u, dt, n, ckpt)
        J.backward()
        return kk.grad

    run(2)                                   # warm-up
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    gk = run(steps)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    finite = bool(torch.isfinite(gk).all())
    g.close()
    del I0
    torch.cuda.empty_cache()
    return wall, finite


def copy_bandwidth(dev, nbytes=1 << 30, reps=5):
    """Achieved bandwidth of a plain device-to-device copy (read + write)."""
    import torch
    a = torch.ones(nbytes // 4, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize(dev)
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / sec / 1e9


def cpu_baseline(seconds, threads=None):
    import torch
    from oracle import step as O
    from paper_2302_04283_amd import workloads as W
    cores = threads or len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    m = 16
    sub = W.make_problem(CONFIG, sub=((56, 56, 56), (m, m, m)))
    S = O.setup(sub)
    dt = O.max_dt(S, sub.cfl)
    rho, u, ka, ks = O.fluid_tensors(sub)
    I = torch.as_tensor(sub.initial_intensity())
    T = torch.as_tensor(sub.T)
    ba = O.beam_angle(S)
    O.step(I, T, S, rho, u, ka, ks, dt, ba)   # warm-up
    n = 0
    t0 = time.perf_counter()
    while True:
        I, T, _, _ = O.step(I, T, S, rho, u, ka, ks, dt, ba)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    rate = m ** 3 * sub.nang * n / el
    return {"value": rate, "unit": "cell-angle updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d steps of a %d^3-cell block of the 128^3 x 162 workload "
                      "(torch float64 on %d host threads, %.1f s)" % (n, m, cores, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--checkpoint-every", type=int, default=10)
    ap.add_argument("--no-context", action="store_true",
                    help="skip the copy-bandwidth and 42/92-direction context rows")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "reference for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 256 * 1024 * 1024
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": 4 * n, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the radiation step is built and timed on a "
              "single MI355X (sharding by space, with one halo exchange per step, is not "
              "built); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2302_04283_amd import rt
    from paper_2302_04283_amd import workloads as W

    dev = torch.device("cuda", 0)
    prob = W.make_problem(CONFIG)
    probe = rt.Grid(prob, rt.RT_F32)
    dt = probe.max_dt(prob.cfl)
    probe.close()
    ncell = prob.ncell
    nang = prob.nang
    K = args.steps
    print("[bench] workload %s: %d cells x %d directions, dt=%.6g, %d warmup + %d timed steps"
          % (CONFIG, ncell, nang, dt, args.warmup, K), file=sys.stderr, flush=True)

    wall32, per32, st32 = time_path(prob, rt.RT_F32, K, args.warmup, dt, dev)
    print("[bench] fp32 done: %.3f ms/step" % (1e3 * wall32 / K), file=sys.stderr, flush=True)
    value = ncell * nang * K / wall32
    # algorithmic bytes per launch: read + write one FP32 intensity per
    # cell-angle, plus per cell rho, u(3), kappa_a, kappa_s (read), T and
    # dT0(4) (read + write): 48 + 16 + 64 = 128 B
    bytes_launch = ncell * (nang * 8 + 128)
    avg = sum(per32) / len(per32)
    achieved = bytes_launch / avg / 1e9
    out = {
        "metric": "cell-angle updates/s (fwd, FP32 intensities + FP64 solve)",
        "value": value,
        "unit": "cell-angle updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall32 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Minkowski Cartesian 128^3 periodic, geodesic level 4 "
                               "(162 directions), random |v|<=0.5, lognormal kappa_a/kappa_s, "
                               "collimated beam; FP32 intensities + FP64 quartic",
                   "cells": ncell, "directions": nang, "dt": dt},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _traffic(bytes_launch),
                     "kernel": "k_march<float, 32, 6> (fused tiled step: transport + coupling "
                               "+ bookkeeping), timed with its finaliser",
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "avg_launch_s": avg},
        "no_root_events": st32["no_root"],
    }
    tr = out["roofline"]["traffic"]
    if tr:
        # the measured HBM bytes over the same launch time, against the peak
        out["roofline"]["traffic_GBs"] = tr / avg / 1e9
        out["roofline"]["traffic_frac"] = tr / avg / 1e9 / HBM_PEAK_GBS
    if not args.no_fp64:
        wall64, per64, _ = time_path(prob, rt.RT_F64, K, args.warmup, dt, dev)
        print("[bench] fp64 done: %.3f ms/step" % (1e3 * wall64 / K), file=sys.stderr, flush=True)
        v64 = ncell * nang * K / wall64
        avg64 = sum(per64) / len(per64)
        b64 = ncell * (nang * 16 + 128)
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * wall64 / K,
                       "achieved_GBs": b64 / avg64 / 1e9, "speedup_fp32_over_fp64": value / v64}
    if not args.no_adjoint:
        precs = [(rt.RT_F32, "fwd_adjoint")] + ([] if args.no_fp64 else [(rt.RT_F64, "fwd_adjoint_fp64")])
        for prec, key in precs:
            wall_fa, finite = time_fwd_adjoint(prob, prec, K, args.checkpoint_every, dt, dev)
            print("[bench] %s done: %.3f ms/step" % (key, 1e3 * wall_fa / K), file=sys.stderr,
                  flush=True)
            out[key] = {"value": ncell * nang * K / wall_fa, "unit": "cell-angle updates/s",
                        "ms_per_step": 1e3 * wall_fa / K,
                        "checkpoint_every": args.checkpoint_every,
                        "gradients_finite": finite,
                        "functional": "luminosity through the upper x face; gradients "
                                      "wrt kappa_a, kappa_s, T0 and I0"}
        if "fwd_adjoint_fp64" in out:
            out["fwd_adjoint"]["speedup_fp32_over_fp64"] = (out["fwd_adjoint"]["value"] /
                                                            out["fwd_adjoint_fp64"]["value"])
    if not args.no_context:
        # a plain device-to-device copy (the STREAM-like ceiling) and the
        # paper's GPU benchmark angle counts on the same 128^3 grid
        out["copy_GBs"] = copy_bandwidth(dev)
        shapes = {}
        for lev in (2, 3):
            p2 = W.make_problem(CONFIG, nlev=lev)
            g2 = rt.Grid(p2, rt.RT_F32)
            dt2 = g2.max_dt(p2.cfl)
            g2.close()
            w2, _, _ = time_path(p2, rt.RT_F32, 20, 3, dt2, dev)
            shapes["%d directions" % p2.nang] = {"value": p2.ncell * p2.nang * 20 / w2,
                                                  "ms_per_step": 1e3 * w2 / 20}
        out["paper_shapes_fp32"] = shapes
        # two-stage integrator alone (tiled kernel, two launches per step)
        p2s = W.make_problem(CONFIG)
        p2s.integrator = 2
        w2s, _, _ = time_path(p2s, rt.RT_F32, 10, 2, dt, dev)
        out["two_stage_fp32"] = {"value": ncell * nang * 10 / w2s, "ms_per_step": 1e3 * w2s / 10,
                                 "integrator": 2, "kernel": "tiled"}
        # the production scheme's options: two-stage integrator and the
        # optical-depth-aware flux (general kernel), same 128^3 x 162 grid
        p3 = W.make_problem(CONFIG)
        p3.integrator, p3.tau_coeff = 2, 5.0
        w3, _, _ = time_path(p3, rt.RT_F32, 10, 2, dt, dev)
        out["two_stage_tau_fp32"] = {"value": ncell * nang * 10 / w3, "ms_per_step": 1e3 * w3 / 10,
                                     "integrator": 2, "tau_coeff": 5.0, "kernel": "general"}
        # radiation-dominated velocity substitute (general kernel) and the
        # hand-over of dT0 to the gas (one thread per cell)
        p4 = W.make_problem(CONFIG)
        p4.rad_velocity = 1
        w4, _, _ = time_path(p4, rt.RT_F32, 10, 2, dt, dev)
        out["rad_velocity_fp32"] = {"value": ncell * nang * 10 / w4, "ms_per_step": 1e3 * w4 / 10,
                                    "kernel": "general",
                                    "gas_update_ms": 1e3 * time_gas_update(p4, dev, 20)}
        # the same box on the latitude-longitude grid, 8 x 16 directions (tiled)
        p5 = W.make_problem(CONFIG)
        p5.latlong = (8, 16)
        w5, _, _ = time_path(p5, rt.RT_F32, 20, 2, dt, dev)
        out["latlong_8x16_fp32"] = {"value": ncell * 128 * 20 / w5, "ms_per_step": 1e3 * w5 / 20}
        # Kerr-Schild, 128 x 64 x 128 cells, 162 directions (general kernel)
        p6 = W.make_problem("c3")
        g6 = rt.Grid(p6, rt.RT_F32, dev.index or 0)
        dt6 = g6.max_dt(p6.cfl)
        g6.close()
        w6, _, _ = time_path(p6, rt.RT_F32, 10, 2, dt6, dev)
        out["kerr_schild_128x64x128_fp32"] = {"value": p6.ncell * p6.nang * 10 / w6,
                                              "ms_per_step": 1e3 * w6 / 10, "kernel": "general"}
        # the same with MAPR angular fluxes
        p6.ang_recon = 2
        w7, _, _ = time_path(p6, rt.RT_F32, 10, 2, dt6, dev)
        out["kerr_schild_mapr_fp32"] = {"value": p6.ncell * p6.nang * 10 / w7,
                                        "ms_per_step": 1e3 * w7 / 10, "kernel": "general"}
        print("[bench] context done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        # the same oracle on one host thread (a third of the sample time)
        one = cpu_baseline(args.cpu_seconds / 3.0, threads=1)
        out["cpu_baseline"]["one_thread"] = {"value": one["value"], "sample": one["sample"]}
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
