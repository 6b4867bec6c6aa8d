"""GPU parity of pruned grids (Sec. 3.6) against the oracle: the kept-cell
masks bit for bit, the preconditioner on the induced cell graph, and the full
step with pruned grids.  At the full 32-frame size (16..128^3) the masks of
sampled transitions are compared bit for bit and the preconditioned gradient
is checked through the residual of (I + lambda L_S)^2 on every level."""
import numpy as np
import pytest
import torch

import synth
from oracle import precond as PC
from oracle import prune as PR
from oracle import sequence as S
from paper_2509_18097_amd import _lib as L
from paper_2509_18097_amd.problem import HyperParams, Problem
from _gpu import assert_rel, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def _pack(masks, res):
    """Oracle masks ([level] of boolean [r, r, r]) in the library's bit layout
    (levels in order, ceil(r^3 / 32) words each, cell c at bit c & 31 of word
    c >> 5) as int32 words."""
    words = []
    for mk, r in zip(masks, res):
        bits = np.zeros(-(-r ** 3 // 32) * 32, dtype=np.uint64)
        bits[:r ** 3] = np.asarray(mk, bool).reshape(-1)
        w = (bits.reshape(-1, 32) << np.arange(32, dtype=np.uint64)).sum(axis=1)
        words.append(w.astype(np.uint32))
    return np.concatenate(words).view(np.int32)


def _unpack(words, res):
    w = np.asarray(words).view(np.uint32).astype(np.uint64)
    out, off = [], 0
    for r in res:
        nw = -(-r ** 3 // 32)
        bits = (w[off:off + nw, None] >> np.arange(32, dtype=np.uint64)) & 1
        out.append(bits.reshape(-1)[:r ** 3].astype(bool).reshape(r, r, r))
        off += nw
    return out


def _points(seed, frames, n):
    rng = np.random.default_rng(seed)
    p = np.concatenate([rng.normal(0.0, 0.35, (frames, 3, n // 2)),
                        rng.uniform(-1.2, 1.2, (frames, 3, n - n // 2))], axis=2)
    p[0, :, :3] = [[-1.0, 1.0, 0.0], [1.0, -1.0, 0.0], [0.0, 0.5, 1.0]]   # faces of the cube
    return p.astype(np.float32)


@pytest.mark.parametrize("res,halo,span", [((1, 3, 5, 8), 3, 2), ((4, 12, 32), 1, 2),
                                           ((8, 16, 64), 3, 1), ((7, 33), 2, 3), ((16,), 0, 2)])
def test_mask_bit_exact(res, halo, span):
    require_gpu()
    pts = _points(sum(res) + halo, 5, 300)
    mask, active = L.prune_mask(dev(pts), res, span=span, halo=halo)
    mask, active = host(mask), host(active)
    ref = PR.stack_masks(pts, res, halo, span)
    assert mask.shape[0] == len(ref) == 5 - span + 1
    for b, ms in enumerate(ref):
        np.testing.assert_array_equal(mask[b], _pack(ms, res), err_msg=f"stack {b}")
        assert active[b].tolist() == [int(m.sum()) for m in ms]


def test_mask_no_points_and_all_points():
    require_gpu()
    res = (4, 8)
    empty = torch.zeros((2, 3, 0), dtype=torch.float32, device="cuda")
    mask, active = L.prune_mask(empty, res)
    assert not host(mask).any() and not host(active).any()
    # a point in every cell of the coarsest level keeps every cell there
    c = -1.0 + (np.arange(4) + 0.5) / 2.0
    g = np.stack(np.meshgrid(c, c, c, indexing="ij")).reshape(3, -1)
    mask, active = L.prune_mask(dev(np.stack([g, g]).astype(np.float32)), res, halo=0)
    assert host(active)[0, 0] == 64


def _rand_masks(rng, res, p):
    return [rng.random((r, r, r)) < p for r in res]


@pytest.mark.parametrize("res,batch", [((4, 8, 12, 16), 2), ((5, 7), 1), ((32,), 1)])
def test_precondition_pruned_matches_oracle(res, batch):
    require_gpu()
    rng = np.random.default_rng(len(res) + batch)
    lams = [0.25 * 1.5 ** l for l in range(len(res))]
    g = rng.normal(size=(batch, L.grid_size(res))).astype(np.float32)
    masks = [_rand_masks(rng, res, 0.7 if b == 0 else 0.35) for b in range(batch)]
    words = np.stack([_pack(m, res) for m in masks])
    out = host(L.precondition_pruned(dev(g), res, lams, dev(words), batch=batch))
    for b in range(batch):
        ref = PR.apply_levels_masked(g[b], res, lams, masks[b])
        off = 0
        for r in res:
            sl = slice(off, off + 3 * r ** 3)
            assert_rel(out[b, sl], ref[sl], 1e-5, f"stack {b} R={r}")
            off += 3 * r ** 3
        keep = PR.packed_mask(masks[b], res)
        assert np.all(out[b, ~keep] == 0.0)


def test_full_mask_equals_box_cg():
    require_gpu()
    res = (4, 8, 16)
    lams = [0.25, 0.375, 0.5625]
    g = synth.grid_stack(3, res, std=1.0)
    words = _pack([np.ones((r, r, r), bool) for r in res], res)
    a = host(L.precondition_pruned(dev(g), res, lams, dev(words)))
    b = host(L.precondition(dev(g), res, lams, method="cg"))
    np.testing.assert_allclose(a, b, rtol=1e-6, atol=1e-7 * np.abs(b).max())
    assert_rel(a, PC.apply_levels(g, res, lams), 1e-5, "box")


def test_step_pruned_matches_oracle():
    require_gpu()
    res = (4, 8, 16)
    seq = synth.deforming_sequence(seed=5, frames=4, n=600, subdiv=1)
    T = 3
    theta0 = np.random.default_rng(6).normal(0, 0.01, (T, L.grid_size(res))).astype(np.float32)
    hp = HyperParams(e_max=10)
    prob = Problem(dev(seq.points), res, template=dev(seq.template), edges=dev(seq.edges),
                   hp=hp, params=dev(theta0), precond="cg", prune_halo=1)
    masks = PR.stack_masks(seq.points, res, halo=1, span=2)
    got = host(prob.prune_mask)
    for t in range(T):
        np.testing.assert_array_equal(got[t], _pack(masks[t], res))
    keep = np.stack([PR.packed_mask(masks[t], res) for t in range(T)])
    theta_p = np.where(keep, theta0, 0.0).astype(np.float32)
    np.testing.assert_array_equal(host(prob.params), theta_p)      # pruned values zeroed
    prob.step(0)
    torch.cuda.synchronize()
    phat, xhat = host(prob.buffer("phat")), host(prob.buffer("xhat"))
    grad, pgrad = host(prob.buffer("grad")), host(prob.buffer("pgrad"))
    z = np.zeros_like(theta_p, dtype=np.float64)
    r = S.step(seq.points, seq.template, seq.edges, res, theta_p, z, z, 0, S.Hyper(e_max=10),
               phat32=phat, xhat32=xhat, grad_override=grad, pgrad_override=pgrad, masks=masks)
    assert_rel(grad, r.grad, 1e-5, "dL/dG")
    assert_rel(pgrad, r.pgrad, 1e-5, "pruned preconditioned")
    assert np.all(pgrad[~keep] == 0.0)
    theta = host(prob.params)
    assert np.max(np.abs(theta - r.theta)) <= 1e-5 * max(S.Hyper().schedule(len(res))[0])
    for e in range(1, 4):
        prob.step(e)
    assert np.all(host(prob.params)[~keep] == 0.0)
    assert np.all(host(prob.m)[~keep] == 0.0) and np.all(host(prob.v)[~keep] == 0.0)


@pytest.fixture(scope="module")
def headline():
    require_gpu()
    seq = synth.deforming_sequence(seed=0, frames=32, n=50_000, subdiv=6)
    res = (16, 32, 64, 128)
    pts = dev(seq.points)
    mask, active = L.prune_mask(pts, res, span=2, halo=3)
    return seq, res, pts, host(mask), host(active)


def test_headline_masks_sampled(headline):
    seq, res, _, mask, active = headline
    assert mask.shape[0] == 31
    for t in (0, 17, 30):
        ms = PR.stack_masks(seq.points[t:t + 2], res, halo=3, span=2)[0]
        np.testing.assert_array_equal(mask[t], _pack(ms, res), err_msg=f"transition {t + 1}")
        assert active[t].tolist() == [int(m.sum()) for m in ms]
    kept = active.sum() / (31 * sum(r ** 3 for r in res))
    assert 0.0 < kept < 0.5           # the paper: more than half of the parameters removed


def test_headline_precondition_residual(headline):
    """(I + lambda L_S)^2 applied to the GPU's result gives back g on the kept
    cells (the a-priori count's A-norm tolerance 1e-7 bounds the residual),
    zero on the pruned ones; on one transition."""
    seq, res, _, mask, _ = headline
    lams = [0.25 * 1.5 ** l for l in range(len(res))]
    g = synth.grid_stack(7, res, std=1.0)
    out = host(L.precondition_pruned(dev(g), res, lams, dev(mask[5])))
    ms = _unpack(mask[5], res)
    off = 0
    for r, lam, mk in zip(res, lams, ms):
        keep = mk.reshape(-1)
        a = PR.induced_laplacian(r, mk) * lam
        for c in range(3):
            sl = slice(off + c * r ** 3, off + (c + 1) * r ** 3)
            x = out[sl].astype(np.float64)
            assert np.all(x[~keep] == 0.0)
            y = x[keep] + a @ x[keep]
            back = y + a @ y
            gk = g[sl].astype(np.float64)[keep]
            assert np.linalg.norm(back - gk) <= 1e-4 * np.linalg.norm(gk), f"R={r} c={c}"
        off += 3 * r ** 3


def test_step_pruned_with_empty_tiles():
    """A compact point set in a box of levels up to 64^3, so that most
    2048-cell conjugate-gradient tiles hold no kept cell: the step's launches
    cover only the kept tiles (the list built at creation), with the tile skip,
    the reductions of spans without a kept tile and the partial-sum zeroing
    all exercised.  The preconditioned gradient against the oracle (Eq. 3 on
    the kept cells' graph) and bitwise against pdg_precondition_pruned, which
    launches every tile."""
    require_gpu()
    res = (4, 16, 32, 64)
    seq = synth.deforming_sequence(seed=11, frames=3, n=800, subdiv=1)
    shift = np.array([0.35, -0.3, 0.2], np.float32)[None, :, None]
    pts = (0.18 * seq.points + shift).astype(np.float32)
    tmpl = (0.18 * seq.template + shift[0]).astype(np.float32)
    T = 2
    theta0 = np.random.default_rng(12).normal(0, 0.01, (T, L.grid_size(res))).astype(np.float32)
    prob = Problem(dev(pts), res, template=dev(tmpl), edges=dev(seq.edges),
                   hp=HyperParams(e_max=10), params=dev(theta0), precond="cg", prune_halo=1)
    masks = PR.stack_masks(pts, res, halo=1, span=2)
    keep = np.stack([PR.packed_mask(masks[t], res) for t in range(T)])
    # most tiles of the 32^3 and 64^3 levels hold no kept cell
    off = 3 * (4 ** 3 + 16 ** 3)
    for r in (32, 64):
        cells = keep[0, off:off + r ** 3]
        tiles = cells.reshape(-1, 2048).any(axis=1)
        assert tiles.sum() < 0.5 * tiles.size, (r, tiles.sum(), tiles.size)
        off += 3 * r ** 3
    theta_p = np.where(keep, theta0, 0.0).astype(np.float32)
    prob.step(0)
    torch.cuda.synchronize()
    phat, xhat = host(prob.buffer("phat")), host(prob.buffer("xhat"))
    grad, pgrad = host(prob.buffer("grad")), host(prob.buffer("pgrad"))
    z = np.zeros_like(theta_p, dtype=np.float64)
    r = S.step(pts, tmpl, seq.edges, res, theta_p, z, z, 0, S.Hyper(e_max=10),
               phat32=phat, xhat32=xhat, grad_override=grad, pgrad_override=pgrad, masks=masks)
    assert_rel(grad, r.grad, 1e-5, "dL/dG")
    assert_rel(pgrad, r.pgrad, 1e-5, "pruned preconditioned (kept tiles only)")
    assert np.all(pgrad[~keep] == 0.0)
    lams = [0.25 * 1.5 ** l for l in range(len(res))]
    full = host(L.precondition_pruned(dev(grad), res, lams, prob.prune_mask, batch=T))
    np.testing.assert_array_equal(pgrad, full)
    theta = host(prob.params)
    assert np.max(np.abs(theta - r.theta)) <= 1e-5 * max(S.Hyper().schedule(len(res))[0])


PAPER_RES = tuple(2 * l - 1 for l in range(1, 11))    # the paper's grid: L = 10, R = 2l - 1


def test_six_channel_step_pruned_paper_grid():
    """The paper's configuration: six-channel cells [z; t] (Eq. 4-7) on pruned
    grids (Sec. 3.6) over R = 1, 3, .., 19.  A compact point set with a one-cell
    halo prunes the outer cells of the finer levels; the pruned values of all
    six channels start and stay at zero, and the step matches the oracle
    stage by stage (gradient, the preconditioner of both halves on the kept
    cells' graph, Adam)."""
    require_gpu()
    res = PAPER_RES
    seq = synth.deforming_sequence(seed=41, frames=4, n=700, subdiv=2)
    pts = (0.45 * seq.points).astype(np.float32)
    tmpl = (0.45 * seq.template).astype(np.float32)
    T = 3
    P6 = L.grid_size(res, 6)
    theta0 = np.random.default_rng(42).normal(0, 0.05, (T, P6)).astype(np.float32)
    print("six-channel pruned step, R = 1..19", flush=True)
    prob = Problem(dev(pts), res, template=dev(tmpl), edges=dev(seq.edges),
                   hp=HyperParams(e_max=10), params=dev(theta0), precond="cg", prune_halo=1,
                   channels=6)
    masks = PR.stack_masks(pts, res, halo=1, span=2)
    got = host(prob.prune_mask)
    for t in range(T):
        np.testing.assert_array_equal(got[t], _pack(masks[t], res))
    keep = np.stack([PR.packed_mask(masks[t], res, channels=6) for t in range(T)])
    assert 0.03 < keep.mean() < 0.9, keep.mean()         # most cells of the finer levels pruned
    theta_p = np.where(keep, theta0, 0.0).astype(np.float32)
    np.testing.assert_array_equal(host(prob.params), theta_p)
    prob.step(1)
    torch.cuda.synchronize()
    phat, xhat = host(prob.buffer("phat")), host(prob.buffer("xhat"))
    grad, pgrad = host(prob.buffer("grad")), host(prob.buffer("pgrad"))
    z = np.zeros_like(theta_p, dtype=np.float64)
    r = S.step(pts, tmpl, seq.edges, res, theta_p, z, z, 1, S.Hyper(e_max=10),
               phat32=phat, xhat32=xhat, grad_override=grad, pgrad_override=pgrad, masks=masks,
               channels=6, workers=4)
    assert_rel(grad, r.grad, 1e-5, "dL/dG (six channels)")
    assert_rel(pgrad, r.pgrad, 1e-5, "pruned preconditioned (six channels)")
    assert np.all(pgrad[~keep] == 0.0)
    eta_max = max(S.Hyper().schedule(len(res))[0])
    assert np.max(np.abs(host(prob.params) - r.theta)) <= 1e-5 * eta_max
    for e in range(2, 5):
        prob.step(e, use_graph=True)
    torch.cuda.synchronize()
    assert np.all(host(prob.params)[~keep] == 0.0)
    assert np.all(host(prob.m)[~keep] == 0.0) and np.all(host(prob.v)[~keep] == 0.0)
    assert np.isfinite(prob.terms()["loss"])
