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
BF16_MFMA_PEAK_TFLOPS = 2500.0     # dense
FP32_VALU_PEAK_TFLOPS = 157.3     # vector FP32, an FMA counted as two flops
PAIR_OPS = 8          # 3 sub + 3 mul + 2 add per pair under the difference-form contract
PAIR_MFMA_FLOPS = 32  # one output of a K = 16 bf16 MFMA
# HBM bytes per launch from two rocprofv3 PMC runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0,
# factors from a 1 GiB copy; mean over the last 8 of 11 launches), recorded in
# profiles/nn_screen_c2_bf16_dct.md for the kernel source whose SHA-256 starts
# with the given prefix; reported only while the source is unchanged.
PMC_TRAFFIC = {
    "nn_screen_kernel": ("paper_2509_18097_amd/csrc/chamfer_screen.hip", "e4f10a87f7e5f3f5",
                         (2 * 314922.03125 + 207658.4609375) * 1024),
}


def pmc_traffic(kernel):
    import hashlib
    if kernel not in PMC_TRAFFIC:
        return None
    path, digest, nbytes = PMC_TRAFFIC[kernel]
    with open(os.path.join(ROOT, path), "rb") as f:
        if not hashlib.sha256(f.read()).hexdigest().startswith(digest):
            return None
    return round(nbytes)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--subdiv", type=int, default=6, choices=(4, 6),
                    help="template icosphere subdivisions (6: 40,962 vertices, 4: 2,562)")
    ap.add_argument("--chamfer", default="bf16", choices=("fp32", "bf16", "fp32cull"),
                    help="bf16: matrix-core screen + exact re-rank (same indices as fp32)")
    ap.add_argument("--precond", default="dct", choices=("cg", "dct"),
                    help="dct: exact spectral solve; cg: conjugate gradients, float64 dots")
    ap.add_argument("--prune", type=int, default=None, metavar="HALO",
                    help="pruned grids for the timed step: kept cells = occupied + HALO-cell "
                         "cube (the paper: 3); needs --precond cg")
    ap.add_argument("--optimize-template", action="store_true",
                    help="optimise X_0 too in the timed step (Eq. 9-10, Sec. 3.6)")
    ap.add_argument("--paper-grid", action="store_true",
                    help="the timed step on the paper's grid: six-channel cells, R = 2l - 1, L = 10")
    ap.add_argument("--keyframe", type=int, default=0,
                    help="X_0 at this frame, propagated both ways (Sec. 3.3); 0: forward only")
    ap.add_argument("--variants", default="fp32:cg,bf16:cg,fp32:dct,fp32cull:dct",
                    help="other chamfer:precond forms to time on the same GPU ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stages", action="store_true", help="skip the per-stage timing")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timings beside the step (six-channel deform, keyframe, "
                         "mesh preconditioner, pruned grids)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--serve", type=int, default=256, metavar="R",
                    help="also serve the first R requests of the 256-request Poisson stream "
                         "(4 requests/s, 20 iterations each); 0 skips, 256 is the full stream")
    ap.add_argument("--serve-load", type=float, default=3.0, metavar="X",
                    help="serve the same requests a second time with arrivals X times as "
                         "frequent (offered load above 1); 1 skips")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single-pair, precision (200k x 200k) and differentiation "
                         "(1M x 1M forward + backward) workloads")
    ap.add_argument("--serve-only", action="store_true", help="skip the sequence benchmark")
    ap.add_argument("--serve-slots", type=int, default=32,
                    help="maximum requests resident and iterating at once")
    ap.add_argument("--serve-executor", default="streams", choices=("streams", "batch", "classes"),
                    help="streams: each request's own graph on 4 streams; batch: one batched "
                         "iteration of all resident requests per round; classes: one batch "
                         "and stream per size class")
    return ap.parse_args()


def make_problem(subdiv, chamfer, precond, prune_halo=None, optimize_template=False, keyframe=0,
                 paper_grid=False):
    import torch
    import synth
    from paper_2509_18097_amd.problem import HyperParams, Problem
    seq = synth.deforming_sequence(seed=0, frames=FRAMES, n=NPTS, subdiv=subdiv)
    prob = Problem(torch.from_numpy(seq.points).cuda(), CAYLEY_RES if paper_grid else RES,
                   template=torch.from_numpy(seq.template).cuda(),
                   edges=torch.from_numpy(seq.edges).cuda(), hp=HyperParams(e_max=50),
                   chamfer_mode=chamfer, precond=precond, prune_halo=prune_halo,
                   optimize_template=optimize_template, keyframe=keyframe,
                   channels=6 if paper_grid else 3)
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
    """Per-stage times inside real iterations: each rep runs the stages in
    step order as the full step runs them (the last being "precond_adam", the
    preconditioner with Adam fused into its last pass where it can), with an
    event recorded between consecutive stages on the stream they are
    enqueued on (torch's current stream), so every stage sees the state an
    iteration gives it (e.g. the nearest-neighbour screen is warm started
    from the previous iteration's assignment, not from its own).  The
    preconditioner and Adam are also timed alone ("precond", "adam")."""
    import torch
    st = torch.cuda.current_stream()
    names = ("warp", "nn", "loss", "grad", "scatter", "precond_adam")
    if getattr(prob, "template_m", None) is not None:
        names += ("template",)
    for name in names:                   # warm
        prob.stage(name)
    torch.cuda.synchronize()
    out = {name: 0.0 for name in names}
    t0 = screen_tiles(prob)              # only the NN stage advances the counter
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        ev[0].record(st)
        for k, name in enumerate(names):
            prob.stage(name)
            ev[k + 1].record(st)
        torch.cuda.synchronize()
        for k, name in enumerate(names):
            out[name] += ev[k].elapsed_time(ev[k + 1]) / reps
    if t0 is not None:
        key = "nn_mfma" if prob.chamfer_mode == "bf16" else "nn_pair_units"
        out[key] = (screen_tiles(prob) - t0) / reps
    alone = ("precond", "adam")
    out.update({name: 0.0 for name in alone})
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(alone) + 1)]
        ev[0].record(st)
        for k, name in enumerate(alone):
            prob.stage(name)
            ev[k + 1].record(st)
        torch.cuda.synchronize()
        for k, name in enumerate(alone):
            out[name] += ev[k].elapsed_time(ev[k + 1]) / reps
    return out


def screen_tiles(prob):
    """Matrix-core products (32 x 32 x 16 bf16 MFMAs) the screen has issued so
    far (bf16 mode), or the 1,024-pair units of distances the culled float32
    search has evaluated (fp32cull mode), else None."""
    if prob.chamfer_mode not in ("bf16", "fp32cull"):
        return None
    if prob.keyframe > 0:
        return sum(int(ch.buffer("screen_tiles").item())
                   for ch in (prob.branch(0), prob.branch(1)) if ch is not None)
    return int(prob.buffer("screen_tiles").item())


def nn_pairs(prob):
    """Pair evaluations of one NN stage: both directions of every Chamfer term."""
    T, N, V = prob.T, prob.n, prob.V
    return 2 * T * N * N + 2 * T * N * V


def cg_bytes(prob):
    """Algorithmic HBM bytes of one preconditioner stage: the copy of the raw
    gradient (8 B/value), and per solve an init pass (12 B/value) plus per
    iteration 12 B (kernel A: read r, p; write p') + 20 B (kernel B: read p',
    x, r; write x, r) per value of every system still iterating.  With pruned
    grids the iterations count only the kept cells (what a solve on the kept
    set alone must move)."""
    T = prob.T
    total = 8 * T * prob.P
    kept = getattr(prob, "kept_cells", None) if prob.prune_mask is not None else None
    for l, r in enumerate(prob.res):
        lam = prob.hp.lambda0 * prob.hp.lambda_growth ** l
        kappa = 1.0 + 12.0 * lam         # a-priori CG count (as the library computes it)
        rho = (math.sqrt(kappa) - 1.0) / (math.sqrt(kappa) + 1.0)
        k = math.ceil(math.log(2.0 / 1e-7) / -math.log(rho))
        cells = T * prob.channels * r ** 3
        it_cells = cells if kept is None else 3 * int(kept[:, l].sum().item())
        total += 2 * (12 * cells + k * 32 * it_cells)
    return total


def dct_stage_bytes(prob):
    """Algorithmic HBM bytes of one DCT preconditioner stage: three passes per
    level of R <= 128 (forward plane, pencil, inverse plane), each reading and
    writing every value once (24 B per grid value), six for R > 128 (48 B);
    R = 1 levels are skipped.  The R = 16, 32, 64 and 128 levels use fast
    transforms and are bound by these bytes."""
    T = prob.T
    return sum((24 if r <= 128 else 48) * T * prob.channels * r ** 3
               for r in prob.res if r > 1)


def roofline(prob, stages, chamfer, precond):
    """Roofline of the nearest-neighbour kernel (the NN stage is exactly one
    launch of it; the largest per-step kernel share in the committed
    rocprofv3 summary) and, second, of the preconditioner stage (several
    launches, reported as one unit)."""
    nn_ms, pre_ms = stages["nn"], stages["precond"]
    pairs = nn_pairs(prob)
    if chamfer == "bf16":
        # the matrix-core work actually issued: each wave counts its own
        # 32 x 32 x 16 products (32,768 flops, 1,024 candidate-query pairs);
        # `brute_force_pairs_per_launch` is the pair count the exact result
        # stands for, of which the box cull and the waves' own tests skip most
        mfma = stages["nn_mfma"]
        screened = mfma * 1024
        a = mfma * 1024 * PAIR_MFMA_FLOPS / (nn_ms * 1e-3) / 1e12
        nn = {"bound": "mfma", "achieved": round(a, 2), "peak": BF16_MFMA_PEAK_TFLOPS,
              "unit": "TFLOP/s", "frac": round(a / BF16_MFMA_PEAK_TFLOPS, 4),
              "traffic": pmc_traffic("nn_screen_kernel"),
              "kernel": "nn_screen_kernel", "mfma_per_launch": int(mfma),
              "pairs_screened_per_launch": int(screened),
              "brute_force_pairs_per_launch": pairs,
              "screened_fraction": round(screened / pairs, 4), "launch_ms": round(nn_ms, 4)}
    elif chamfer == "fp32cull":
        # the distances actually evaluated after the box cull, each at the
        # exact pair's cost
        ev = stages["nn_pair_units"] * 1024
        a = ev * PAIR_OPS / (nn_ms * 1e-3) / 1e12
        nn = {"bound": "alu", "achieved": round(a, 2), "peak": round(VALU_PEAK_TOPS, 2),
              "unit": "TFLOP/s", "frac": round(a / VALU_PEAK_TOPS, 4), "traffic": None,
              "kernel": "nn_cull_kernel", "pairs_evaluated_per_launch": int(ev),
              "brute_force_pairs_per_launch": pairs,
              "evaluated_fraction": round(ev / pairs, 4), "launch_ms": round(nn_ms, 4)}
    else:
        a = pairs * PAIR_OPS / (nn_ms * 1e-3) / 1e12
        nn = {"bound": "alu", "achieved": round(a, 2), "peak": round(VALU_PEAK_TOPS, 2),
              "unit": "TFLOP/s", "frac": round(a / VALU_PEAK_TOPS, 4), "traffic": None,
              "kernel": "nn_exact_kernel", "pairs_per_launch": pairs,
              "launch_ms": round(nn_ms, 4)}
    if precond == "dct":
        b = dct_stage_bytes(prob)
        a = b / (pre_ms * 1e-3) / 1e9
        pre = {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(a / HBM_PEAK_GBS, 4), "traffic": None,
               "kernel": "DCT stage: plane, pencil, plane kernels per level (fast transforms "
                         "at R = 16, 32, 64, 128)", "bytes_per_stage": b, "stage_ms": round(pre_ms, 4)}
    else:
        b = cg_bytes(prob)
        a = b / (pre_ms * 1e-3) / 1e9
        pre = {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(a / HBM_PEAK_GBS, 4), "traffic": None,
               "kernel": "cg_a_kernel/cg_b_kernel (+ reductions)", "bytes_per_stage": b,
               "stage_ms": round(pre_ms, 4), "pruned": prob.prune_mask is not None}
    return nn, pre


CAYLEY_RES = tuple(2 * l - 1 for l in range(1, 11))   # the paper's grid: L = 10, R = 2l - 1
CAYLEY_N = 1_000_000


def time_cayley6(reps=10):
    """Six-channel cells (Sec. 3.3, Eq. 4-7) on the paper's grid (L = 10,
    R = 1, 3, ..., 19): pdg_deform and pdg_deform_backward (grid and position
    adjoints) of 1,000,000 points uniform in [-1, 1]^3, grid values N(0, 0.2^2).
    The grid (0.48 MB) stays in L2, so the forward is bound by the vector ALU:
    per point and level 48 interpolation FMAs (6 channels x 8 corners) and 16
    flops of weights, plus ~40 flops of the rotation."""
    import numpy as np
    import torch
    import synth
    from paper_2509_18097_amd import _lib as L
    res, n = CAYLEY_RES, CAYLEY_N
    rng = np.random.default_rng(0)
    g = torch.from_numpy(synth.grid_stack(0, res, std=0.2, channels=6)).cuda()
    x = torch.from_numpy(rng.uniform(-1.0, 1.0, (3, n)).astype(np.float32)).cuda()
    q = torch.from_numpy(rng.normal(size=(3, n)).astype(np.float32)).cuda()
    out = torch.empty_like(x)
    for _ in range(2):
        L.deform(g, x, res, out=out, channels=6)
        L.deform_backward(g, x, q, res, channels=6)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(st)
    for _ in range(reps):
        L.deform(g, x, res, out=out, channels=6)
    ev[1].record(st)
    for _ in range(reps):
        L.deform_backward(g, x, q, res, channels=6)
    ev[2].record(st)
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) / reps
    bwd = ev[1].elapsed_time(ev[2]) / reps
    flops = n * (len(res) * (2 * 48 + 16) + 40)
    a = flops / (fwd * 1e-3) / 1e12
    return {"workload": "six-channel Cayley cells, paper grid L = 10 (R = 1..19), "
                        "1,000,000 points in [-1,1]^3",
            "fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4),
            "points_per_s_fwd": round(n / (fwd * 1e-3), 1),
            "points_per_s_fwd_bwd": round(n / ((fwd + bwd) * 1e-3), 1),
            "fwd_roofline": {"bound": "alu", "achieved": round(a, 2), "peak": FP32_VALU_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(a / FP32_VALU_PEAK_TFLOPS, 4),
                             "traffic": None, "kernel": "warp6_kernel",
                             "flops_per_launch": flops}}


def time_mesh_precond(seq, reps=10):
    """The mesh-vertex preconditioner (I + 16 L)^-2 (Sec. 3.2, 3.6) on the
    template (40,962 vertices, 122,880 edges, degrees <= 6): one application
    of a built plan (the Chebyshev series of t^-2, tol 1e-8, eight terms per
    launch on LDS-resident vertex parts).  Roofline: the float64 vectors'
    traffic of one term (the neighbourhood gather at 3 x 8 B per vertex and
    edge end, the own v_j, v_{j-1} reads and v_{j+1} write: 3 x 8 B x (2E +
    3V)) per term, against HBM, as if every term went through memory."""
    import numpy as np
    import torch
    from paper_2509_18097_amd import _lib as L
    edges = torch.from_numpy(np.ascontiguousarray(seq.edges, dtype=np.int32)).cuda()
    v = seq.template.shape[1]
    e = edges.shape[1]
    dmax = int(np.bincount(np.asarray(seq.edges).reshape(-1), minlength=v).max())
    g = torch.from_numpy(np.random.default_rng(0).normal(size=(3, v)).astype(np.float32)).cuda()
    out = torch.empty_like(g)
    plan = L.MeshPlan(edges, v, dmax, 16.0)
    plan.apply(g, out=out)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        plan.apply(g, out=out)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    per_term = 3 * 8 * (2 * e + 3 * v)
    gbs = per_term * (plan.terms - 1) / (ms * 1e-3) / 1e9
    k = L.mesh_partition(seq.edges, v)[4]
    res = {"workload": f"template mesh, {v} vertices, {e} edges, lambda 16",
           "ms": round(ms, 4), "max_degree": dmax, "series_terms": plan.terms,
           "vertex_parts": plan.parts, "terms_per_launch": k,
           "launches": 1 + -(-(plan.terms - 1) // k) if plan.parts else plan.terms,
           "effective_GBs": round(gbs, 1)}
    plan.close()
    return res


def time_pruned(subdiv, chamfer, steps=6, reps=5):
    """Pruned grids (Sec. 3.6) on the headline sequence: kept-cell masks of
    every transition from the two frames it connects with a three-cell halo,
    and the full step with the conjugate-gradient preconditioner on the kept
    cells' graph (tiles without a kept cell skipped).  The dense step with the
    same preconditioner is timed beside it."""
    import torch
    from paper_2509_18097_amd import _lib as L
    out = {}
    for name, halo in (("dense_cg", None), ("pruned_cg", 3)):
        seq, prob = make_problem(subdiv, chamfer, "cg", prune_halo=halo)
        ms, _ = time_steps(prob, steps, 2)
        st = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            prob.stage("precond")
        b.record(st)
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": round(ms, 4), "precond_ms": round(a.elapsed_time(b) / reps, 4)}
        if halo is not None:
            kept = prob.kept_cells.sum().item()
            cells = prob.T * sum(r ** 3 for r in RES)
            a.record(st)
            for _ in range(reps):
                L.prune_mask(prob.points, RES, 2, halo)
            b.record(st)
            torch.cuda.synchronize()
            out[name].update({"halo": halo, "kept_fraction": round(kept / cells, 4),
                              "kept_fraction_per_level": [
                                  round(v, 4) for v in (prob.kept_cells.sum(0).double().cpu()
                                                        / (prob.T * torch.tensor(RES) ** 3)).tolist()],
                              "mask_ms": round(a.elapsed_time(b) / reps, 4)})
        prob.close()
        del prob
        torch.cuda.empty_cache()
    return out


def time_template(subdiv, chamfer, precond, steps=10, reps=5):
    """The headline step with X_0 optimised as well (Eq. 9-10, Sec. 3.6): the
    TEMPLATE stage adds L_mesh = CD_R(X_0, P_0) with its gradient (40,962
    vertices against 50,000 points), the mesh preconditioner (the Chebyshev
    series of its plan) and Adam on X_0."""
    import torch
    _, prob = make_problem(subdiv, chamfer, precond, optimize_template=True)
    ms, _ = time_steps(prob, steps, 2)
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        prob.stage("template")
    b.record(st)
    torch.cuda.synchronize()
    out = {"ms_per_step": round(ms, 4), "iterations_per_s": round(1000.0 / ms, 4),
           "template_stage_ms": round(a.elapsed_time(b) / reps, 4)}
    prob.close()
    del prob
    torch.cuda.empty_cache()
    return out


def time_two_way(subdiv, chamfer, precond, keyframe, steps=10):
    """The headline sequence with X_0 at a middle frame, propagated both ways
    (Sec. 3.3, end): a backward chain of `keyframe` transitions and a forward
    chain of the rest, one problem, one graph per step."""
    import torch
    _, prob = make_problem(subdiv, chamfer, precond, keyframe=keyframe)
    ms, _ = time_steps(prob, steps, 2)
    out = {"keyframe": keyframe, "ms_per_step": round(ms, 4),
           "iterations_per_s": round(1000.0 / ms, 4)}
    prob.close()
    del prob
    torch.cuda.empty_cache()
    return out


def time_step6(subdiv, chamfer, precond, steps=10):
    """The headline sequence on the paper's own grid: six-channel cells [z; t]
    (Eq. 4-7) on the 2l - 1 schedule with L = 10 (R = 1, 3, .., 19), full step
    (rotation-aware warps and adjoints, both halves preconditioned)."""
    import torch
    import synth
    from paper_2509_18097_amd.problem import HyperParams, Problem
    seq = synth.deforming_sequence(seed=0, frames=FRAMES, n=NPTS, subdiv=subdiv)
    prob = Problem(torch.from_numpy(seq.points).cuda(), CAYLEY_RES,
                   template=torch.from_numpy(seq.template).cuda(),
                   edges=torch.from_numpy(seq.edges).cuda(), hp=HyperParams(e_max=50),
                   chamfer_mode=chamfer, precond=precond, channels=6)
    ms, _ = time_steps(prob, steps, 2)
    out = {"grid": "six-channel cells, R = 2l - 1, L = 10", "ms_per_step": round(ms, 4),
           "iterations_per_s": round(1000.0 / ms, 4)}
    prob.close()
    del prob
    torch.cuda.empty_cache()
    return out


def time_keyframe(seq, reps=20):
    """Keyframe selection (Sec. 3.5, Eq. 19-20) over the sequence's frames:
    one bit per occupied 128^3 voxel and frame, population counts, the
    weighted argmax.  Algorithmic HBM bytes: the points once (12 B each) and
    the bitsets written and read once (2 x 256 KiB per frame)."""
    import torch
    from paper_2509_18097_amd import _lib as L
    pts = torch.from_numpy(seq.points).cuda()
    key, _ = L.keyframe(pts)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        L.keyframe(pts)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    f, n = pts.shape[0], pts.shape[2]
    nbytes = 12 * f * n + 2 * f * 128 ** 3 // 8
    return {"workload": f"{f} frames x {n} points", "ms": round(ms, 4),
            "key": int(key.item()), "gb_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}


def time_pair(chamfer="fp32", precond="dct", iters=50):
    """Single frame pair: 4,096 points on the unit sphere against their
    displacement by 0.1 sin(2 pi x) plus N(0, 0.002^2), grids 8/16/32 x 3
    channels from zero, `iters` Adam iterations of the full step (graph
    replay), timed from zero parameters."""
    import numpy as np
    import torch
    import synth
    from paper_2509_18097_amd.problem import HyperParams, Problem
    src, tgt = synth.pair_on_sphere(seed=0, n=4096)
    pts = torch.from_numpy(np.stack([src, tgt])).cuda()
    prob = Problem(pts, (8, 16, 32), hp=HyperParams(e_max=iters), chamfer_mode=chamfer,
                   precond=precond)
    prob.step(0, use_graph=True)            # captures the graph
    for t in (prob.params, prob.m, prob.v):
        t.zero_()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for e in range(iters):
        prob.step(e, use_graph=True)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    last = prob.terms()["loss"]
    prob.close()
    return {"workload": "single frame pair, 4,096 points on the unit sphere, grids 8/16/32^3 "
                        f"x 3 ch, {iters} Adam iterations from zero grids",
            "chamfer": chamfer, "precond": precond, "iterations": iters,
            "ms_total": round(ms, 4), "iterations_per_s": round(iters / (ms * 1e-3), 2),
            "loss_last": last}


def _argmin_f64(q, c, chunk=256):
    """Nearest index of every column of q among the columns of c, float64
    difference form, first index on ties (torch, on the device): the float64
    reference the float32 neighbour contract is measured against."""
    import torch
    out = []
    cd = c.double()
    for i in range(0, q.shape[1], chunk):
        d = q[:, i:i + chunk].double().T[:, :, None] - cd[None, :, :]
        out.append(torch.argmin((d * d).sum(dim=1), dim=1))
    return torch.cat(out)


def time_precision(n=200_000, reps=3, sample=20_000):
    """200,000 points U[-1,1]^3 against the same jittered by N(0, 0.01^2), both
    directions (Eq. 11-13): the float32 brute force and the bf16 screen with
    exact re-rank, timed as one pdg_chamfer call each (the screen's call
    includes the Morton sorts and packs of both sets, cold, no warm start);
    their indices compared in full; a sample of queries compared with the
    float64 argmin (flips) and the relative error of the loss terms against
    the float64 assignment."""
    import numpy as np
    import torch
    import synth
    from paper_2509_18097_amd import _lib as L
    p, q = synth.cloud_pair_cube(seed=0, n=n)
    a, b = torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda()
    st = torch.cuda.current_stream()
    out = {"workload": f"{n:,} points U[-1,1]^3 vs the same + N(0, 0.01^2), both directions",
           "brute_force_pairs": 2 * n * n}
    res = {}
    for mode in ("fp32", "bf16", "fp32cull"):
        L.chamfer(a, b, 5.56, mode)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            r = L.chamfer(a, b, 5.56, mode)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[mode] = r
        pps = 2 * n * n / (ms * 1e-3)
        ent = {"ms": round(ms, 4), "brute_force_pairs_per_s": round(pps, 1)}
        if mode == "fp32":
            a_ = pps * PAIR_OPS / 1e12
            ent["roofline"] = {"bound": "alu", "achieved": round(a_, 2),
                               "peak": round(VALU_PEAK_TOPS, 2), "unit": "TFLOP/s",
                               "frac": round(a_ / VALU_PEAK_TOPS, 4), "kernel": "nn_exact_kernel"}
        out[mode] = ent
    out["bf16_speedup"] = round(out["fp32"]["ms"] / out["bf16"]["ms"], 2)
    # the same tile cull without matrix cores: what the cull alone buys
    out["fp32cull_speedup"] = round(out["fp32"]["ms"] / out["fp32cull"]["ms"], 2)
    out["bf16_speedup_over_fp32cull"] = round(out["fp32cull"]["ms"] / out["bf16"]["ms"], 2)
    for mode in ("bf16", "fp32cull"):
        out[f"index_mismatches_{mode}_vs_fp32"] = int((res["fp32"][1] != res[mode][1]).sum().item() +
                                                      (res["fp32"][2] != res[mode][2]).sum().item())
    out["loss_fp32"] = res["fp32"][0].cpu().tolist()
    out["loss_bf16"] = res["bf16"][0].cpu().tolist()
    # float64 reference on a sample of each direction's queries
    g = torch.Generator(device="cpu")
    g.manual_seed(0)
    rep = {"sampled_queries_per_direction": sample}
    for name, qs, cs, nn in (("a_to_b", a, b, res["fp32"][1]), ("b_to_a", b, a, res["fp32"][2])):
        idx = torch.randperm(qs.shape[1], generator=g)[:sample].cuda()
        qq = qs[:, idx]
        n64 = _argmin_f64(qq, cs)
        n32 = nn[idx].long()
        d32 = ((qq.double() - cs[:, n32].double()) ** 2).sum(0)
        d64 = ((qq.double() - cs[:, n64].double()) ** 2).sum(0)
        ent = {"flips_fp32_vs_fp64": int((n32 != n64).sum().item())}
        for alpha in (5.56, 0.0):
            t32 = (torch.exp(-alpha * d32) * d32).sum().item()
            t64 = (torch.exp(-alpha * d64) * d64).sum().item()
            ent[f"loss_rel_err_alpha_{alpha}"] = abs(t32 - t64) / t64
        rep[name] = ent
    out["fp64_reference"] = rep
    return out


RES5 = (16, 32, 64, 128, 256)


def time_differentiation(reps=3, n=1_000_000):
    """Forward and backward through the torch.autograd functions with the
    hand-written adjoints: warp of 1,000,000 points U[-1,1]^3 through a
    5-level grid stack 16^3..256^3 (N(0, 0.01^2) values), Chamfer (bf16
    screen, exact re-rank) against 1,000,000 independent points, backward to
    all 57.5M grid values."""
    import torch
    import synth
    from paper_2509_18097_amd import autograd as AG
    grids = torch.from_numpy(synth.grid_stack(0, RES5, std=0.01)).cuda().requires_grad_()
    x = torch.from_numpy(synth.uniform_cube(1, n)).cuda()
    t = torch.from_numpy(synth.uniform_cube(2, n)).cuda()
    st = torch.cuda.current_stream()

    def fwd():
        out = AG.deform(grids, x, RES5)
        loss, _, _ = AG.chamfer(out, t, mode="bf16")
        return loss

    loss = fwd()
    loss.sum().backward()
    torch.cuda.synchronize()
    tf = tb = 0.0
    for _ in range(reps):
        grids.grad = None
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(st)
        loss = fwd()
        ev[1].record(st)
        loss.sum().backward()
        ev[2].record(st)
        torch.cuda.synchronize()
        tf += ev[0].elapsed_time(ev[1]) / reps
        tb += ev[1].elapsed_time(ev[2]) / reps
    return {"workload": f"5-level grid stack 16..256^3 x 3 ch (57.5M values), {n:,} queries "
                        f"chained into Chamfer (bf16 screen) against {n:,} targets",
            "forward_ms": round(tf, 3), "backward_ms": round(tb, 3),
            "seconds_per_forward_backward": round((tf + tb) * 1e-3, 5),
            "loss": loss.detach().cpu().tolist()}


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


def serve_requests(count):
    """The first `count` requests of the 256-request Poisson stream (4/s;
    point counts log-uniform in [2k, 200k]; 8..64 frames; 3-5 levels by point
    count; 20 iterations each), their inputs drawn on the GPU up front so they
    are resident before the stream starts."""
    import torch
    import synth
    from paper_2509_18097_amd.serve import poisson_requests
    stream = synth.request_stream(seed=0, count=256)[:count]
    t = time.perf_counter()
    reqs = []
    for i in range(0, len(stream), 32):
        reqs += poisson_requests(stream[i:i + 32], iterations=20, device="cuda")
        print(f"serve: {len(reqs)}/{len(stream)} request inputs drawn", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return reqs, time.perf_counter() - t


# size classes of the batched executor: bounds on points x frames (the stream's
# requests span 16,000 to 12,800,000)
SERVE_BUCKETS = (2e5, 1.5e6, 5e6)


def serve(reqs, chamfer, precond, slots=32, rate_scale=1.0, executor="streams"):
    """Serve the requests with continuous batching under an HBM budget of 60%
    of free memory; arrival times divided by `rate_scale` (1: the stream's
    4 requests/s).  executor "batch": every round one batched iteration of all
    resident requests (one launch of the screen and Chamfer terms over all
    their jobs); "classes": one such batch per size class, each on a stream
    of its own; "streams": each request's own graph replayed on 4 streams."""
    import dataclasses
    import torch
    from paper_2509_18097_amd.serve import BatchExecutor, GpuExecutor, Server
    reqs = [dataclasses.replace(r, arrival=r.arrival / rate_scale) for r in reqs]
    free, _ = torch.cuda.mem_get_info()
    if executor == "batch":
        ex = BatchExecutor(chamfer_mode=chamfer, precond=precond)
    elif executor == "classes":
        ex = BatchExecutor(chamfer_mode=chamfer, precond=precond, buckets=SERVE_BUCKETS)
    else:
        ex = GpuExecutor(chamfer_mode=chamfer, precond=precond, streams=4)
    st = Server(ex, budget_bytes=int(0.6 * free), max_slots=slots).run(reqs)
    out = st.summary()
    out.update({"executor": executor, "stream_requests": len(reqs), "iterations_per_request": 20,
                "arrival_rate_per_s": 4.0 * rate_scale,
                "budget_bytes": int(0.6 * free), "chamfer": chamfer, "precond": precond,
                "max_slots": slots,
                "load": round(st.makespan / st.arrival_span, 3) if st.arrival_span > 0 else None})
    if executor.startswith("batch"):
        out["batches_built"] = ex.batches_built
        out["size_classes"] = len(ex.streams)
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}


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
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): the path would "
              "shard its transitions across GPUs, which is not run here.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.serve_only:
        reqs, gen_s = serve_requests(args.serve)
        out = serve(reqs, args.chamfer, args.precond, args.serve_slots,
                    executor=args.serve_executor)
        out["input_generation_s"] = round(gen_s, 2)
        print(json.dumps({"metric": METRIC, "serving": out}))
        return
    if args.prune is not None and args.precond != "cg":
        sys.exit("--prune needs --precond cg (the DCT solve needs the full box)")
    seq, prob = make_problem(args.subdiv, args.chamfer, args.precond, args.prune,
                             args.optimize_template, args.keyframe, args.paper_grid)
    torch.cuda.synchronize()
    ms, wall = time_steps(prob, args.steps, args.warmup)
    value = 1000.0 / ms
    terms = prob.terms()
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
                               f"{'/'.join(str(r) for r in prob.res)}^3 x {prob.channels} ch per "
                               f"transition",
                   "frames": FRAMES, "points_per_frame": NPTS, "template_verts": prob.V,
                   "template_edges": prob.E, "grid_res": list(prob.res), "chamfer": args.chamfer,
                   "precond": args.precond, "graph_replay": True,
                   **({"prune_halo": args.prune} if args.prune is not None else {}),
                   **({"optimize_template": True} if args.optimize_template else {}),
                   **({"keyframe": args.keyframe} if args.keyframe else {}),
                   **({"cells": "six-channel, R = 2l - 1, L = 10"} if args.paper_grid else {})},
        "loss_last_step": terms["loss"],
    }
    if stages:
        result["stages_ms"] = {k: round(v, 4) for k, v in stages.items()}
        result["roofline"], result["roofline_other"] = roofline(prob, stages, args.chamfer,
                                                                args.precond)
    T_, V_ = prob.T, prob.V
    prob.close()
    del prob
    torch.cuda.empty_cache()
    variants = {}
    for v in [x for x in args.variants.split(",") if x]:
        ch, pc = v.split(":")
        _, vp = make_problem(args.subdiv, ch, pc)
        vms, _ = time_steps(vp, max(3, args.steps // 2), 2)
        variants[v] = {"ms_per_step": round(vms, 4), "iterations_per_s": round(1000.0 / vms, 4)}
        if not args.no_stages:
            vst = time_stages(vp, reps=2)
            nn_r, pre_r = roofline(vp, vst, ch, pc)
            variants[v]["stages_ms"] = {k: round(x, 4) for k, x in vst.items()}
            variants[v]["nn_roofline"] = {k: nn_r[k] for k in ("bound", "achieved", "peak", "unit",
                                                               "frac", "kernel")}
            variants[v]["precond_roofline"] = {k: pre_r[k] for k in ("bound", "achieved", "peak",
                                                                     "unit", "frac", "kernel")}
        vp.close()
        del vp
        torch.cuda.empty_cache()
    if variants:
        result["variants"] = variants
    if not args.no_configs:
        result["single_pair"] = time_pair("fp32", args.precond)
        result["single_pair_bf16"] = time_pair("bf16", args.precond)
        result["precision"] = time_precision()
        result["differentiation"] = time_differentiation()
        torch.cuda.empty_cache()
    if not args.no_extras:
        result["cayley6"] = time_cayley6()
        result["keyframe"] = time_keyframe(seq)
        result["mesh_precond"] = time_mesh_precond(seq)
        result["pruned"] = time_pruned(args.subdiv, args.chamfer)
        result["template_opt"] = time_template(args.subdiv, args.chamfer, args.precond)
        result["two_way"] = time_two_way(args.subdiv, args.chamfer, args.precond, FRAMES // 2)
        result["step6"] = time_step6(args.subdiv, args.chamfer, args.precond)
    if args.serve > 0:
        reqs, gen_s = serve_requests(args.serve)
        result["serving"] = serve(reqs, args.chamfer, args.precond, args.serve_slots,
                                  executor=args.serve_executor)
        result["serving"]["input_generation_s"] = round(gen_s, 2)
        if args.serve_load > 1.0:
            result["serving_overload"] = serve(reqs, args.chamfer, args.precond, args.serve_slots,
                                               rate_scale=args.serve_load,
                                               executor=args.serve_executor)
        del reqs
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        workers = min(16, os.cpu_count() or 1)
        dt = cpu_baseline(seq, workers)
        result["cpu_baseline"] = {
            "value": round(1.0 / (dt * T_), 6), "unit": "iterations/s", "cores": workers,
            "host_cpu_count": os.cpu_count(), "kind": "oracle",
            "sample": f"one of {T_} transitions (all stages at full size: 50k points, "
                      f"{V_}-vertex template, 16..128^3 grids, DCT preconditioner), "
                      f"{dt:.1f} s, scaled x{T_}"}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
