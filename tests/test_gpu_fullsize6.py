"""Parity at full size on the paper's own grid, in the configuration bench.py
times for it (`--paper-grid`): the 32-frame x 50,000-point sequence with the
40,962-vertex template on six-channel cells [z; t] with R = 1, 3, .., 19
(L = 10), BF16-screened Chamfer, DCT preconditioner, graph replay.  Two
iterations are run (the first moves the grids off zero); the second is checked
against the oracle on sampled outputs, each oracle stage fed the GPU's float32
inputs to that stage."""
import numpy as np
import pytest
import torch

import synth
from oracle import adam as A
from oracle import cayley as CY
from oracle import chamfer as C
from oracle import precond as P
from oracle import sequence as S
from paper_2509_18097_amd.problem import HyperParams, Problem
from _gpu import dev, host, require_gpu

pytestmark = pytest.mark.gpu
RES = tuple(2 * l - 1 for l in range(1, 11))
LS = 1.0 / len(RES)


@pytest.fixture(scope="module")
def run6():
    require_gpu()
    seq = synth.deforming_sequence(seed=0, frames=32, n=50_000, subdiv=6)
    prob = Problem(dev(seq.points), RES, template=dev(seq.template), edges=dev(seq.edges),
                   hp=HyperParams(e_max=50), chamfer_mode="bf16", precond="dct", channels=6)
    print("full-size six-channel sequence: step 0", flush=True)
    prob.step(0, use_graph=True)
    torch.cuda.synchronize()
    theta1, m1, v1 = host(prob.params), host(prob.m), host(prob.v)
    print("full-size six-channel sequence: step 1", flush=True)
    prob.step(1, use_graph=True)
    torch.cuda.synchronize()
    out = {k: host(prob.buffer(k)) for k in ("phat", "xhat", "grad", "pgrad", "gphat", "gxhat",
                                              "lam")}
    out["nn"] = {k: host(v) for k, v in prob.nn().items()}
    out["theta2"] = host(prob.params)
    prob.close()
    return seq, theta1, m1, v1, out


def _rel(got, ref):
    d = np.asarray(got, np.float64) - ref
    return max(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300),
               np.max(np.abs(d)) / max(np.max(np.abs(ref)), 1e-300))


def _off_kinks(x, res, margin=1e-4):
    """Samples away from every cell-centre plane (where the position Jacobian is
    one-sided and float32 and float64 may take different sides)."""
    ok = np.ones(x.shape[1], bool)
    for r in res:
        if r == 1:
            continue
        u = (x.astype(np.float64) + 1.0) * r / 2.0 - 0.5
        ok &= np.all(np.abs(u - np.round(u)) > margin, axis=0)
    return ok


def test_six_channel_warps_and_neighbours_sampled(run6):
    seq, th, _, _, o = run6
    rng = np.random.default_rng(2)
    for t in (0, 14, 30):
        idx = rng.choice(50_000, 400, replace=False)
        src = seq.points[t][:, idx]
        ref = CY.warp6(th[t], RES, src, LS)
        assert np.all(np.abs(o["phat"][t][:, idx] - ref) <=
                      1e-5 * np.abs(ref - src).max() + 4e-7 * np.abs(ref))
        vi = rng.choice(40_962, 400, replace=False)
        src = o["xhat"][t][:, vi]
        ref = CY.warp6(th[t], RES, src, LS)
        assert np.all(np.abs(o["xhat"][t + 1][:, vi] - ref) <=
                      1e-5 * np.abs(ref - src).max() + 4e-7 * np.abs(ref))
        tgt = seq.points[t + 1]
        for q, c, key in ((o["phat"][t], tgt, "pt_ab"), (o["xhat"][t + 1], tgt, "tm_ab")):
            qi = rng.choice(q.shape[1], 100, replace=False)
            assert np.array_equal(o["nn"][key][t][qi], C.nn_fp32(q[:, qi], c, workers=8)), (t, key)


def test_six_channel_gradients_sampled(run6):
    seq, th, _, _, o = run6
    T = 31
    lams = [0.25 * 1.5 ** l for l in range(len(RES))]
    errs = {}
    for t in (0, 19, 30):
        if t < T - 1:
            # one step of the reverse sweep from the GPU's later adjoint
            ok = _off_kinks(o["xhat"][t + 1], RES)
            lam = o["gxhat"][t] + CY.position_adjoint6(th[t + 1], RES, o["xhat"][t + 1],
                                                       o["lam"][t + 1], LS)
            errs[f"chain adjoint t={t} ({(~ok).sum()} on kinks masked)"] = \
                _rel(o["lam"][t][:, ok], lam[:, ok])
        ref = CY.grid_adjoint6(th[t], RES, seq.points[t], o["gphat"][t], LS) + \
            CY.grid_adjoint6(th[t], RES, o["xhat"][t], o["lam"][t], LS)
        errs[f"dL/dG t={t}"] = _rel(o["grad"][t], ref)
        errs[f"precond t={t}"] = _rel(o["pgrad"][t],
                                      P.apply_levels(o["grad"][t], RES, lams, "dct", channels=6))
    for k, v in errs.items():
        print(f"{k}: {v:.2e}", flush=True)
    assert max(errs.values()) <= 1e-5, errs


def test_six_channel_adam_full(run6):
    _, th, m, v, o = run6
    etas = [5e-3 * 1.1 ** l for l in range(len(RES))]
    off = 0
    for l, r in enumerate(RES):
        sl = slice(off, off + 6 * r ** 3)
        ref, _, _ = A.update(th[:, sl], m[:, sl], v[:, sl], o["pgrad"][:, sl], etas[l], 2)
        assert np.max(np.abs(o["theta2"][:, sl] - ref)) <= 1e-5 * etas[l]
        off += 6 * r ** 3
