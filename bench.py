#!/usr/bin/env python3
"""Deform-and-match benchmark on one MI355X.

Workload (the plain method at full size): a 32-frame sequence of 50,000
points per frame on a deforming ellipsoid (axes 1, 0.6, 0.4; smooth
random-Fourier motion, 8 modes, amplitude 0.05; noise N(0, 0.003^2)), a
6-times-subdivided icosphere template (40,962 vertices, 122,880 edges) and
4 grid levels 16^3 .. 128^3 per transition (31 transitions).  One step is one
full iteration of the method: warp of points and template chain, bidirectional
robust Chamfer (point and template terms), isometry, confidence weights, the
gradient scatter into the grids, the (I + lambda L)^-2 preconditioner and Adam.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Inputs are resident in HBM before the timed region;
the step is replayed from a captured HIP graph.  The headline value is
iterations per second of the whole step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "deform+Chamfer iterations/sec at 50k pts/frame; p50/p99 served-solve latency"
FRAMES, NPTS, RES = 32, 50_000, (16, 32, 64, 128)
# MI355X: 256 CUs x 128 FP32 VALU lanes per clock x 2.4 GHz = 78.6e12 FP32
# lane operations per second (the published 157.3 TFLOP/s counts an FMA as 2);
# HBM3E 8 TB/s.
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
PAIR_OPS = 8          # 3 sub + 3 mul + 2 add per pair under the difference-form contract


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--subdiv", type=int, default=6, choices=(4, 6),
                    help="template icosphere subdivisions (6: 40,962 vertices, 4: 2,562)")
    ap.add_argument("--chamfer", default="fp32", choices=("fp32", "bf16"))
    ap.add_argument("--precond", default="cg", choices=("cg", "dct"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stages", action="store_true", help="skip the per-stage timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def make_problem(subdiv, chamfer, precond):
    import torch
    import synth
    from paper_2509_18097_amd.problem import HyperParams, Problem
    seq = synth.deforming_sequence(seed=0, frames=FRAMES, n=NPTS, subdiv=subdiv)
    prob = Problem(torch.from_numpy(seq.points).cuda(), RES,
                   template=torch.from_numpy(seq.template).cuda(),
                   edges=torch.from_numpy(seq.edges).cuda(), hp=HyperParams(e_max=50),
                   chamfer_mode=chamfer, precond=precond)
    return seq, prob


def time_steps(prob, steps, warmup):
    import torch
    st = torch.cuda.current_stream()
    e_max = prob.hp.e_max
    for e in range(warmup):
        prob.step(e % (e_max + 1), use_graph=True)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall = time.perf_counter()
    t0.record(st)
    for k in range(steps):
        prob.step((warmup + k) % (e_max + 1), use_graph=True)
    t1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    return t0.elapsed_time(t1) / steps, wall


def time_stages(prob, reps=3):
    """Each stage alone, `reps` times, bracketed by events on the stream it is
    enqueued on (torch's current stream)."""
    import torch
    from paper_2509_18097_amd import _lib as L
    st = torch.cuda.current_stream()
    out = {}
    for name in L.STAGES:
        prob.stage(name)                 # warm
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            prob.stage(name)
        b.record(st)
        torch.cuda.synchronize()
        out[name] = a.elapsed_time(b) / reps
    return out


def nn_pairs(prob):
    """Pair evaluations of one NN stage: both directions of every Chamfer term."""
    T, N, V = prob.T, prob.n, prob.V
    return 2 * T * N * N + 2 * T * N * V


def cg_bytes(prob):
    """Algorithmic HBM bytes of one preconditioner stage: the copy of the raw
    gradient (8 B/value), and per solve an init pass (12 B/value) plus per
    iteration 12 B (kernel A: read r, p; write p') + 20 B (kernel B: read p',
    x, r; write x, r) per value of every system still iterating."""
    T = prob.T
    total = 8 * T * prob.P
    for l, r in enumerate(prob.res):
        lam = prob.hp.lambda0 * prob.hp.lambda_growth ** l
        kappa = 1.0 + 12.0 * lam         # a-priori CG count (as the library computes it)
        rho = (math.sqrt(kappa) - 1.0) / (math.sqrt(kappa) + 1.0)
        k = math.ceil(math.log(2.0 / 1e-7) / -math.log(rho))
        cells = T * 3 * r ** 3
        total += 2 * (12 * cells + k * 32 * cells)
    return total


def cpu_baseline(seq, workers):
    """The oracle on one transition (t = 1) of the same workload, all stages,
    full sizes; scaled to iterations/s of the 31-transition step."""
    import numpy as np
    from oracle import adam as A
    from oracle import chamfer as C
    from oracle import precond as P
    from oracle import sequence as S
    from oracle import warp as W
    hp = S.Hyper(e_max=50)
    etas, lams = hp.schedule(len(RES))
    ls = 1.0 / len(RES)
    P_ = 3 * sum(r ** 3 for r in RES)
    theta = np.zeros(P_)
    t0 = time.perf_counter()
    p0, p1 = seq.points[0], seq.points[1]
    phat = W.warp(theta, RES, p0, ls).astype(np.float32)
    xhat = W.warp(theta, RES, seq.template, ls).astype(np.float32)
    na = C.nn_fp32(phat, p1, workers=workers)
    nb = C.nn_fp32(p1, phat, workers=workers)
    ta = C.nn_fp32(xhat, p1, workers=workers)
    tb = C.nn_fp32(p1, xhat, workers=workers)
    cd = [C.direction_loss(phat, p1, na), C.direction_loss(p1, phat, nb),
          C.direction_loss(xhat, p1, ta), C.direction_loss(p1, xhat, tb)]
    _, g_iso = S.isometry(np.stack([seq.template, xhat]), seq.edges, hp.w_iso)
    gp = C.gradient(phat, p1, na, nb, hp.alpha, 1 / 31, 1 / 31)
    gx = C.gradient(xhat, p1, ta, tb, hp.alpha, 1 / 31, 1 / 31) + g_iso[1]
    grad = W.grid_adjoint(RES, p0, gp, ls) + W.grid_adjoint(RES, seq.template, gx, ls)
    pg = P.apply_levels(grad, RES, lams)
    off = 0
    for l, r in enumerate(RES):
        sl = slice(off, off + 3 * r ** 3)
        A.update(theta[sl], np.zeros(3 * r ** 3), np.zeros(3 * r ** 3), pg[sl], etas[l], 1)
        off += 3 * r ** 3
    dt = time.perf_counter() - t0
    assert all(math.isfinite(c) for c in cd)
    return dt


def copy_calibration():
    import torch
    from paper_2509_18097_amd import _lib as L  # noqa: F401  (loads nothing until used)
    n = 1 << 28                                  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the multi-GPU "
              "sharding of this path is described in DESIGN.md and is not run.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    seq, prob = make_problem(args.subdiv, args.chamfer, args.precond)
    torch.cuda.synchronize()
    ms, wall = time_steps(prob, args.steps, args.warmup)
    value = 1000.0 / ms
    stages = {} if args.no_stages else time_stages(prob)
    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "wall_s_timed": round(wall, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"deforming-ellipsoid sequence, {FRAMES} frames x {NPTS} points, "
                               f"icosphere template {prob.V} verts / {prob.E} edges, grids "
                               f"{'/'.join(str(r) for r in RES)}^3 x 3 ch per transition",
                   "frames": FRAMES, "points_per_frame": NPTS, "template_verts": prob.V,
                   "template_edges": prob.E, "grid_res": list(RES), "chamfer": args.chamfer,
                   "precond": args.precond, "graph_replay": True},
    }
    if stages:
        result["stages_ms"] = {k: round(v, 4) for k, v in stages.items()}
        nn_ms = stages["nn"]
        pre_ms = stages["precond"]
        nn_tflops = nn_pairs(prob) * PAIR_OPS / (nn_ms * 1e-3) / 1e12
        pre_gbs = cg_bytes(prob) / (pre_ms * 1e-3) / 1e9
        nn_roof = {"bound": "alu", "achieved": round(nn_tflops, 3), "peak": round(VALU_PEAK_TOPS, 2),
                   "unit": "TFLOP/s", "frac": round(nn_tflops / VALU_PEAK_TOPS, 4),
                   "traffic": None, "kernel": "nn_exact_kernel",
                   "pairs_per_launch": nn_pairs(prob), "launch_ms": round(nn_ms, 4)}
        pre_roof = {"bound": "hbm", "achieved": round(pre_gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(pre_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "preconditioner stage (cg_a/cg_b)",
                    "bytes_per_stage": cg_bytes(prob), "stage_ms": round(pre_ms, 4)}
        dominant = max(("nn", "precond"), key=lambda k: stages[k])
        result["roofline"] = nn_roof if dominant == "nn" else pre_roof
        result["roofline_other"] = pre_roof if dominant == "nn" else nn_roof
    if not args.no_cpu_baseline:
        workers = min(16, os.cpu_count() or 1)
        dt = cpu_baseline(seq, workers)
        result["cpu_baseline"] = {
            "value": round(1.0 / (dt * prob.T), 6), "unit": "iterations/s", "cores": workers,
            "kind": "oracle",
            "sample": f"one of {prob.T} transitions (all stages at full size: 50k points, "
                      f"{prob.V}-vertex template, 16..128^3 grids, DCT preconditioner), "
                      f"{dt:.1f} s, scaled x{prob.T}"}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
