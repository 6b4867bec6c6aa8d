"""GPU parity of the full step on the paper's own cells [z; t] (Eq. 4-7):
warps x' = R(z^) x + t^ for the points and the template chain, the
rotation-aware reverse sweep and grid gradient (rotation channels from
u = d<g, x'>/dz^, translation channels from g), the preconditioner on each half
of the six channels, Adam; each stage on the GPU's own float32 input."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import cayley as CY
from oracle import precond as PC
from oracle import sequence as S
from paper_2509_18097_amd import _lib as L
from paper_2509_18097_amd.problem import HyperParams, Problem
from _gpu import assert_rel, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def _positions_close(got, ref, src):
    disp = np.max(np.abs(ref - src)) if ref.size else 0.0
    tol = 1e-5 * disp + 8 * 2.0 ** -23 * np.abs(ref) + 1e-12
    assert np.all(np.abs(got - ref) <= tol)


@pytest.mark.parametrize("res,mode,precond", [((3, 8, 13), "fp32", "dct"),
                                              ((1, 3, 5, 7, 9), "bf16", "cg"),
                                              ((4, 16), "bf16", "dct")])
def test_six_channel_step_matches_oracle(res, mode, precond):
    require_gpu()
    seq = synth.deforming_sequence(seed=31, frames=4, n=700, subdiv=2)
    T = 3
    theta0 = np.random.default_rng(32).normal(0, 0.05, (T, L.grid_size(res, 6))).astype(np.float32)
    prob = Problem(dev(seq.points), res, template=dev(seq.template), edges=dev(seq.edges),
                   hp=HyperParams(e_max=10), params=dev(theta0), chamfer_mode=mode,
                   precond=precond, channels=6)
    prob.step(1)
    torch.cuda.synchronize()
    phat, xhat = host(prob.buffer("phat")), host(prob.buffer("xhat"))
    grad, pgrad = host(prob.buffer("grad")), host(prob.buffer("pgrad"))
    z = np.zeros_like(theta0, dtype=np.float64)
    r = S.step(seq.points, seq.template, seq.edges, res, theta0, z, z, 1, S.Hyper(e_max=10),
               phat32=phat, xhat32=xhat, grad_override=grad, pgrad_override=pgrad, channels=6,
               workers=4, precond_method="dct")
    ls = 1.0 / len(res)
    _positions_close(phat, r.phat, seq.points[:-1])
    np.testing.assert_array_equal(xhat[0], seq.template)
    for t in range(1, T + 1):
        _positions_close(xhat[t], CY.warp6(theta0[t - 1], res, xhat[t - 1], ls), xhat[t - 1])
    nn = {k: host(v) for k, v in prob.nn().items()}
    for k, v in r.nn.items():
        np.testing.assert_array_equal(nn[k], v, err_msg=k)
    losses = host(prob.buffer("losses"))
    np.testing.assert_allclose(losses[:T], r.cd_pt, rtol=1e-10, atol=0)
    np.testing.assert_allclose(losses[T:2 * T], r.cd_tm, rtol=1e-10, atol=0)
    assert abs(prob.terms()["loss"] - r.loss) <= 1e-10 * abs(r.loss)
    assert_rel(host(prob.buffer("gphat")), r.g_phat, 1e-5, "dL/dP^")
    assert_rel(grad, r.grad, 1e-5, "dL/dG (six channels)")
    assert_rel(pgrad, r.pgrad, 1e-5, "preconditioned (six channels)")
    eta_max = max(S.Hyper().schedule(len(res))[0])
    assert np.max(np.abs(host(prob.params) - r.theta)) <= 1e-5 * eta_max


def test_six_channel_graph_replay_equals_eager():
    require_gpu()
    res = (3, 8)
    seq = synth.deforming_sequence(seed=33, frames=3, n=500, subdiv=1)
    th = np.random.default_rng(34).normal(0, 0.05, (2, L.grid_size(res, 6))).astype(np.float32)
    a, b = [Problem(dev(seq.points), res, template=dev(seq.template), edges=dev(seq.edges),
                    hp=HyperParams(e_max=10), params=dev(th), chamfer_mode="bf16", channels=6)
            for _ in range(2)]
    for e in range(3):
        a.step(e)
        b.step(e, use_graph=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(a.params), host(b.params))
        assert a.terms() == b.terms()


def test_six_channel_adam_binding():
    require_gpu()
    from oracle import adam as A
    res = (3, 4)
    rng = np.random.default_rng(36)
    th, g = [rng.normal(size=L.grid_size(res, 6)).astype(np.float32) for _ in range(2)]
    lrs = [5e-3, 5.5e-3]
    t, m, v = dev(th), torch.zeros(th.size, device="cuda"), torch.zeros(th.size, device="cuda")
    L.adam(t, m, v, dev(g), res, lrs, 1, channels=6)
    off = 0
    for r, lr in zip(res, lrs):
        sl = slice(off, off + 6 * r ** 3)
        ref, _, _ = A.update(th[sl], 0.0, 0.0, g[sl], lr, 1)
        # the update to 1e-6 of the rate, plus the float32 rounding of the stored value
        assert np.all(np.abs(host(t)[sl] - ref) <= 1e-6 * lr + 2.0 ** -23 * np.abs(ref))
        off += 6 * r ** 3


@pytest.mark.parametrize("method", ["dct", "cg"])
def test_six_channel_precondition_matches_oracle(method):
    require_gpu()
    res = (1, 3, 4, 7, 16)
    lams = [0.25 * 1.5 ** l for l in range(len(res))]
    g = np.random.default_rng(35).normal(size=(2, L.grid_size(res, 6))).astype(np.float32)
    d = L.grid_desc(res, 1.0, 6)
    gt = dev(g)
    nb = ctypes.c_size_t()
    L.check(L.lib().pdg_precondition_workspace(ctypes.byref(d), 2, L.PRECOND_METHODS[method],
                                               ctypes.byref(nb)), "ws")
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
    lam = (ctypes.c_float * L.MAX_LEVELS)(*lams)
    L.check(L.lib().pdg_precondition(ctypes.byref(d), lam, ctypes.c_void_p(gt.data_ptr()), 2,
                                     L.PRECOND_METHODS[method], 0, 1e-7,
                                     ctypes.c_void_p(ws.data_ptr()), nb.value,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "pdg_precondition")
    out = host(gt)
    for b in range(2):
        assert_rel(out[b], PC.apply_levels(g[b], res, lams, "dct", channels=6), 1e-5, f"stack {b}")
