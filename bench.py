#!/usr/bin/env python3
"""Benchmark of the fused radiation step on one MI355X.

Headline workload: Minkowski Cartesian 128^3 periodic box, geodesic level 4
(162 directions), random fluid velocities |v| <= 0.5, lognormal absorption
and scattering, collimated beam; FP32 intensities with the FP64 quartic and
bookkeeping.  A step is one pass of the whole hot path: boundary handling,
reconstruction, spatial and angular fluxes, divergence, primitives, the
|n_0| mask, the implicit coupling with its quartic, four-momentum
bookkeeping and the luminosity.  Inputs are resident in HBM before the timed
region starts.

Prints one JSON line: value = cell-angle updates per second (FP32 path),
plus the plain-FP64 rate, forward + adjoint, the roofline of the step
kernel, the 256 x 128 x 256 x 362 Kerr-Schild torus workload (forward in
FP32 and FP64, forward + adjoint with checkpoints), context rows, and the CPU
oracle's rate on a bounded sample of the workload together with the error
of the timed configurations against it.
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
# non-packed FP32 (packed FP32 is not used) and FP64 vector issue:
# 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6
CONFIG = "c2"
# algorithmic floating-point operations per cell-direction of the one-stage
# step with PLM: transport 32 (per axis a shared upwind face value 6, its
# flux 1, the divergence and the axis sum 2; Q* and I* 5) and coupling 37
# (boost 6, implicit factors 5, the three angle sums 10, the update 6, the
# change and its four bookkeeping sums 10); angular fluxes on a curved
# geometry add 7 (about three edges per direction, each flux formed once)
FLOPS_FLAT = 69
FLOPS_CURVED = 76
KERNEL_SOURCES = {"k_march": ["k_march.hip", "k_tile.h", "k_common.h"],
                  "k_column": ["k_column.hip", "k_transport.h", "k_common.h"]}
# rt_grid_info path codes
KERNEL_NAMES = {0: "general", 1: "tiled", 2: "column"}


def _upload_initial(prob, dtype, dev):
    """The workload's initial intensities on the device in `dtype`; the FP64
    field is generated on the host once per problem object and kept on the
    device (the 256 x 128 x 256 x 362 field takes tens of seconds)."""
    import numpy as np
    import torch
    init = prob.extras.get("dev_init64")
    if init is None:
        init = torch.empty((prob.n[2], prob.n[1], prob.n[0], prob.nang), dtype=torch.float64,
                           device=dev)
        for kr, arr in prob.initial_intensity_slabs(np.float64):
            init[kr[0]:kr[1]] = torch.as_tensor(arr).to(dev)
        prob.extras["dev_init64"] = init
    return init.to(dtype, copy=True)


def _kernel_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2302_04283_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(name, kernel):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current sources of that kernel (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != _kernel_hash(kernel):
        return None
    return d.get("hbm_bytes_per_launch")


def _roofline(kernel_name, kernel, cells, nang, per, flops_per, traffic_file, real_bytes=4):
    """Roofline of one step kernel from its event-timed launches: the ALU
    bound it sits under (algorithmic flops against the vector peak) and its
    position against HBM (algorithmic and measured bytes)."""
    avg = sum(per) / len(per)
    flops = cells * nang * flops_per
    byts = cells * (nang * 2 * real_bytes + 128)
    tr = _traffic(traffic_file, kernel)
    out = {"bound": "alu", "achieved": flops / avg / 1e12, "peak": ALU_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": flops / avg / 1e12 / ALU_PEAK_TFLOPS, "traffic": tr,
           "kernel": kernel_name, "algorithmic_flops_per_launch": flops,
           "avg_launch_s": avg,
           "hbm": {"achieved_GBs": byts / avg / 1e9, "peak_GBs": HBM_PEAK_GBS,
                   "frac": byts / avg / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": byts}}
    if tr:
        out["hbm"]["traffic_GBs"] = tr / avg / 1e9
        out["hbm"]["traffic_frac"] = tr / avg / 1e9 / HBM_PEAK_GBS
    return out


def time_path(prob, precision, steps, warmup, dt, dev):
    import torch
    from paper_2302_04283_amd import rt
    g = rt.Grid(prob, precision, dev.index or 0)
    print("[bench] %s %dx%dx%d x %d: %s kernel" % (
        "fp32" if precision == rt.RT_F32 else "fp64", prob.n[0], prob.n[1], prob.n[2], prob.nang,
        KERNEL_NAMES[g.path]), file=sys.stderr, flush=True)
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
    st["kernel"] = KERNEL_NAMES[g.path]
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


def timed_errors(cfg, precisions, dev, origin, m=12, steps=2, full=None):
    """Error of the timed configuration against the oracle (part of the CPU
    baseline leg): the GPU runs the full grid for `steps` steps, the oracle
    a block of m^3 cells at `origin` plus a halo of two cells per step (the
    PLM reach) evolved with outflow/vacuum edges, and the block is compared:
    e_I = max |dI| / (|I| + 1e-3 max|I|) (the parity tests' norm), e_I_raw =
    max |dI| / |I| over nonzero I, e_T = max |dT| / T."""
    import numpy as np
    import torch
    from oracle import step as O
    from paper_2302_04283_amd import rt
    from paper_2302_04283_amd import workloads as W
    full = full if full is not None else W.make_problem(cfg)
    g = rt.Grid(full, precisions[0], dev.index or 0)
    dt = g.max_dt(full.cfl)
    g.close()
    halo = 2 * steps
    sub = W.make_problem(cfg, sub=(tuple(o - halo for o in origin), (m + 2 * halo,) * 3))
    S = O.setup(sub)
    Io, To, _, _ = O.run(sub, S, sub.initial_intensity(), sub.T, dt, steps)
    sl = slice(halo, halo + m)
    Io, To = Io.numpy()[sl, sl, sl], To.numpy()[sl, sl, sl]
    out = {"block": "%d^3 cells at %s, %d steps of the full grid" % (m, origin, steps)}
    for prec in precisions:
        g = rt.Grid(full, prec, dev.index or 0)
        Ia = _upload_initial(full, g.real_dtype(), dev)
        Ib = torch.empty_like(Ia)
        T = torch.as_tensor(full.T).to(dev)
        args = [torch.as_tensor(x).to(dev) for x in (full.rho, full.u_tet, full.kappa_a, full.kappa_s)]
        for _ in range(steps):
            g.step(Ia, Ib, T, *args, dt)
            Ia, Ib = Ib, Ia
        torch.cuda.synchronize(dev)
        ii = [torch.as_tensor((origin[a] + np.arange(m)) % full.n[a], device=dev) for a in range(3)]
        Ig = Ia[ii[2]][:, ii[1]][:, :, ii[0]].double().cpu().numpy()
        Tg = T[ii[2]][:, ii[1]][:, :, ii[0]].cpu().numpy()
        g.close()
        del Ia, Ib, T, args
        torch.cuda.empty_cache()
        d = np.abs(Ig - Io)
        nz = np.abs(Io) > 0
        out["fp32" if prec == rt.RT_F32 else "fp64"] = {
            "e_I": float((d / (np.abs(Io) + 1e-3 * np.abs(Io).max())).max()),
            "e_I_raw": float((d[nz] / np.abs(Io[nz])).max()),
            "e_T": float((np.abs(Tg - To) / To).max())}
    return out


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
    ap.add_argument("--no-torus", action="store_true",
                    help="skip the 256x128x256x362 Kerr-Schild torus rows")
    ap.add_argument("--torus-steps", type=int, default=20)
    ap.add_argument("--no-context", action="store_true",
                    help="skip the copy-bandwidth and option context rows")
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
    per_sorted = sorted(per32)
    out = {
        "metric": "cell-angle updates/s (fwd, FP32 intensities + FP64 solve)",
        "value": value,
        "unit": "cell-angle updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall32 / K,
        "ms_per_step_median": 1e3 * per_sorted[len(per_sorted) // 2],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Minkowski Cartesian 128^3 periodic, geodesic level 4 "
                               "(162 directions), random |v|<=0.5, lognormal kappa_a/kappa_s, "
                               "collimated beam; FP32 intensities + FP64 quartic",
                   "cells": ncell, "directions": nang, "dt": dt},
        # the step kernel issues VALU instructions at about half the issue
        # ceiling while far below the HBM peak: ALU bound (see the SQ counters)
        "roofline": _roofline("k_march<float, 32, 6> (fused tiled step: transport + coupling "
                              "+ bookkeeping), timed with its finaliser", "k_march", ncell, nang,
                              per32, FLOPS_FLAT, "traffic_k_march_c2.json"),
        "hbm_target_note": "the transport-step target of 60% of HBM peak is not met: the "
                           "fused step is instruction-issue bound (roofline.hbm.frac)",
        "no_root_events": st32["no_root"],
    }
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
    p5 = None
    if not args.no_torus:
        # Kerr-Schild a = 0.9, 256 x 128 x 256 cells, level 6 (362 directions),
        # optically thick torus: forward in FP32 (column kernel) and FP64, and
        # forward + adjoint in FP32 with a checkpoint every 4 steps (5
        # checkpoints, 5 segment states, 4 stored I*, 3 adjoint buffers: 17
        # states of 12.2 GB in 288 GB; in FP64 no checkpoint interval fits)
        p5 = W.make_problem("c5")
        g5 = rt.Grid(p5, rt.RT_F32, 0)
        dt5 = g5.max_dt(p5.cfl)
        g5.close()
        n5 = args.torus_steps
        t5 = {"workload": "Kerr-Schild a=0.9, 256x128x256 (r log-spaced [1.3, 50], theta "
                          "[pi/16, 15pi/16], phi periodic), geodesic level 6 (362 directions), "
                          "optically thick torus (tau up to 100)",
              "cells": p5.ncell, "directions": p5.nang, "dt": dt5, "steps": n5}
        w5, per5, st5 = time_path(p5, rt.RT_F32, n5, 2, dt5, dev)
        print("[bench] torus fp32 done: %.2f ms/step" % (1e3 * w5 / n5), file=sys.stderr, flush=True)
        t5["fp32"] = {"value": p5.ncell * p5.nang * n5 / w5, "ms_per_step": 1e3 * w5 / n5,
                      "ms_per_step_median": 1e3 * sorted(per5)[len(per5) // 2],
                      "no_root_events": st5["no_root"],
                      "roofline": _roofline("k_column<float, 3, true, 2, 0, false, false, false> (fused column step, a "
                                            "column's six direction chunks over two waves: "
                                            "transport + angular fluxes + coupling + "
                                            "bookkeeping)",
                                            "k_column", p5.ncell, p5.nang, per5, FLOPS_CURVED,
                                            "traffic_k_column_c5.json")}
        if not args.no_fp64:
            n64 = max(2, n5 // 4)
            w64, per64, st64 = time_path(p5, rt.RT_F64, n64, 1, dt5, dev)
            print("[bench] torus fp64 done: %.2f ms/step" % (1e3 * w64 / n64), file=sys.stderr,
                  flush=True)
            t5["fp64"] = {"value": p5.ncell * p5.nang * n64 / w64, "ms_per_step": 1e3 * w64 / n64,
                          "steps": n64, "kernel": st64["kernel"],
                          "speedup_fp32_over_fp64": t5["fp32"]["value"] / (p5.ncell * p5.nang * n64 / w64)}
        if not args.no_adjoint:
            wfa, finite = time_fwd_adjoint(p5, rt.RT_F32, n5, 4, dt5, dev)
            print("[bench] torus fwd+adjoint done: %.2f ms/step" % (1e3 * wfa / n5),
                  file=sys.stderr, flush=True)
            t5["fwd_adjoint_fp32"] = {"value": p5.ncell * p5.nang * n5 / wfa,
                                      "ms_per_step": 1e3 * wfa / n5, "checkpoint_every": 4,
                                      "state_buffers": 17,
                                      "state_GB": 4.0 * p5.ncell * p5.nang / 1e9,
                                      "gradients_finite": finite,
                                      "functional": "luminosity through the outer r face; "
                                                    "gradients wrt kappa_a, kappa_s, T0, I0"}
        out["kerr_schild_torus_256x128x256x362"] = t5
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
        p2s.extras["dev_init64"] = prob.extras["dev_init64"]     # the same field
        p2s.integrator = 2
        w2s, _, _ = time_path(p2s, rt.RT_F32, 10, 2, dt, dev)
        out["two_stage_fp32"] = {"value": ncell * nang * 10 / w2s, "ms_per_step": 1e3 * w2s / 10,
                                 "integrator": 2, "kernel": "tiled"}
        # the production scheme's options: two-stage integrator and the
        # optical-depth-aware flux (column kernel), same 128^3 x 162 grid
        p3 = W.make_problem(CONFIG)
        p3.extras["dev_init64"] = prob.extras["dev_init64"]     # the same field
        p3.integrator, p3.tau_coeff = 2, 5.0
        w3, _, st3 = time_path(p3, rt.RT_F32, 10, 2, dt, dev)
        out["two_stage_tau_fp32"] = {"value": ncell * nang * 10 / w3, "ms_per_step": 1e3 * w3 / 10,
                                     "integrator": 2, "tau_coeff": 5.0, "kernel": st3["kernel"]}
        # radiation-dominated velocity substitute (column kernel) and the
        # hand-over of dT0 to the gas (one thread per cell)
        p4 = W.make_problem(CONFIG)
        p4.extras["dev_init64"] = prob.extras["dev_init64"]     # the same field
        p4.rad_velocity = 1
        w4, _, st4 = time_path(p4, rt.RT_F32, 10, 2, dt, dev)
        out["rad_velocity_fp32"] = {"value": ncell * nang * 10 / w4, "ms_per_step": 1e3 * w4 / 10,
                                    "kernel": st4["kernel"],
                                    "gas_update_ms": 1e3 * time_gas_update(p4, dev, 20)}
        # the same box on the latitude-longitude grid, 8 x 16 directions (tiled)
        p5l = W.make_problem(CONFIG)
        p5l.latlong = (8, 16)
        w5l, _, _ = time_path(p5l, rt.RT_F32, 20, 2, dt, dev)
        out["latlong_8x16_fp32"] = {"value": ncell * 128 * 20 / w5l, "ms_per_step": 1e3 * w5l / 20}
        # Kerr-Schild, 128 x 64 x 128 cells, 162 directions, DC and MAPR
        # angular fluxes (column kernel)
        p6 = W.make_problem("c3")
        g6 = rt.Grid(p6, rt.RT_F32, dev.index or 0)
        dt6 = g6.max_dt(p6.cfl)
        g6.close()
        w6, _, st6 = time_path(p6, rt.RT_F32, 10, 2, dt6, dev)
        out["kerr_schild_128x64x128_fp32"] = {"value": p6.ncell * p6.nang * 10 / w6,
                                              "ms_per_step": 1e3 * w6 / 10, "kernel": st6["kernel"]}
        w6d, _, st6d = time_path(p6, rt.RT_F64, 10, 2, dt6, dev)
        out["kerr_schild_128x64x128_fp64"] = {"value": p6.ncell * p6.nang * 10 / w6d,
                                              "ms_per_step": 1e3 * w6d / 10, "kernel": st6d["kernel"]}
        # the same grid with the two-stage integrator (column kernel, two
        # launches per step)
        p6.integrator = 2
        w6s, _, st6s = time_path(p6, rt.RT_F32, 10, 2, dt6, dev)
        out["kerr_schild_128x64x128_two_stage_fp32"] = {
            "value": p6.ncell * p6.nang * 10 / w6s, "ms_per_step": 1e3 * w6s / 10,
            "integrator": 2, "kernel": st6s["kernel"]}
        p6.integrator = 1
        p6.ang_recon = 2
        w7, _, st7 = time_path(p6, rt.RT_F32, 10, 2, dt6, dev)
        out["kerr_schild_mapr_fp32"] = {"value": p6.ncell * p6.nang * 10 / w7,
                                        "ms_per_step": 1e3 * w7 / 10, "kernel": st7["kernel"]}
        # the differentiation workload: Kerr-Schild 64 x 32 x 64 cells, 92
        # directions, 50 steps forward + hand-written adjoint with a
        # checkpoint every 10 steps, FP32 and FP64 (gradient of the outgoing
        # luminosity with respect to kappa_a and the gas temperature)
        p8 = W.make_problem("c4")
        g8 = rt.Grid(p8, rt.RT_F32, dev.index or 0)
        dt8 = g8.max_dt(p8.cfl)
        g8.close()
        c4 = {"workload": "Kerr-Schild a=0.9, 64x32x64, 92 directions, 50 steps, checkpoint every 10",
              "steps": 50, "checkpoint_every": 10}
        for prec8, nm8 in ((rt.RT_F32, "fp32"), (rt.RT_F64, "fp64")):
            w8, fin8 = time_fwd_adjoint(p8, prec8, 50, 10, dt8, dev)
            c4[nm8] = {"value": p8.ncell * p8.nang * 50 / w8, "ms_per_step": 1e3 * w8 / 50,
                       "gradients_finite": fin8}
        c4["speedup_fp32_over_fp64"] = c4["fp32"]["value"] / c4["fp64"]["value"]
        out["kerr_schild_64x32x64_fwd_adjoint"] = c4
        print("[bench] context done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        # the same oracle on one host thread (a third of the sample time)
        one = cpu_baseline(args.cpu_seconds / 3.0, threads=1)
        out["cpu_baseline"]["one_thread"] = {"value": one["value"], "sample": one["sample"]}
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
        # the timed configurations' error against the oracle: a block with
        # beam cells and the periodic seam (128^3 x 162), and a block inside
        # the torus (256 x 128 x 256 x 362, FP32 as timed)
        out["errors"] = {"c2_128cubed": timed_errors("c2", (rt.RT_F32, rt.RT_F64), dev,
                                                       (-4, 56, 56), full=prob)}
        if not args.no_torus:
            out["errors"]["torus_256x128x256x362"] = timed_errors("c5", (rt.RT_F32,), dev,
                                                                  (150, 58, 100), full=p5)
        print("[bench] errors done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
