"""GPU parity of the six-channel cells (Sec. 3.3, Eq. 4-7) against the oracle:
pdg_deform / pdg_deform_backward with channels = 6, including the paper's
2l - 1 resolution schedule (L = 10: R = 1, 3, ..., 19)."""
import numpy as np
import pytest
import torch

import synth
from oracle import cayley as C
from oracle import warp as W
from paper_2509_18097_amd import _lib as L
from _gpu import assert_rel, dev, host, require_gpu

pytestmark = pytest.mark.gpu

PAPER_RES = tuple(2 * l - 1 for l in range(1, 11))
CASES = [((1, 3, 5, 7), 3001, 0), ((8, 16, 32), 4096 + 77, 1), (PAPER_RES, 20_000, 2),
         ((5,), 257, 3)]


def _inputs(res, n, seed, lim=1.1, std=0.2):
    rng = np.random.default_rng(seed)
    g = synth.grid_stack(seed, res, std=std, channels=6)
    x = rng.uniform(-lim, lim, (3, n)).astype(np.float32)
    return g, x


def _off_kinks(x, res):
    """Samples not within rounding of a cell-centre plane or the clamp boundary
    (there float32 and float64 may take different one-sided derivatives)."""
    ok = np.ones(x.shape[1], bool)
    for r in res:
        if r == 1:
            continue
        u = (x.astype(np.float64) + 1.0) * r / 2.0 - 0.5
        ok &= np.all(np.abs(u - np.round(u)) > 1e-4, axis=0)
    return ok


@pytest.mark.parametrize("res,n,seed", CASES)
def test_warp6_matches_oracle(res, n, seed):
    require_gpu()
    g, x = _inputs(res, n, seed)
    print(f"warp6 res={res} n={n}", flush=True)
    out = host(L.deform(dev(g), dev(x), res, channels=6))
    ref = C.warp6(g, res, x, 1.0 / len(res))
    assert np.max(np.abs(out - ref) / (1.0 + np.abs(ref))) <= 4e-6


def test_zero_rotation_equals_translation_warp():
    require_gpu()
    res = (4, 8, 16)
    rng = np.random.default_rng(4)
    t = synth.grid_stack(4, res, std=0.05)
    x = rng.uniform(-1.2, 1.2, (3, 5000)).astype(np.float32)
    parts, off = [], 0
    for r in res:
        n3 = 3 * r ** 3
        parts += [np.zeros(n3, np.float32), t[off:off + n3]]
        off += n3
    g6 = np.concatenate(parts)
    a = host(L.deform(dev(g6), dev(x), res, channels=6))
    b = host(L.deform(dev(t), dev(x), res))
    # R(0) = I: the same float32 translation warp, up to one rounding
    assert np.all(np.abs(a - b) <= 2.0 ** -23 * np.abs(b) + 1e-30)


def test_constant_cells_are_a_rigid_motion():
    require_gpu()
    res = PAPER_RES
    x = np.random.default_rng(5).uniform(-1.3, 1.3, (3, 4000)).astype(np.float32)
    cell = np.array([0.25, -0.5, 0.125, 0.0625, -0.25, 0.5], np.float32)   # exact in float32
    g = np.concatenate([np.repeat(cell, r ** 3) for r in res]).astype(np.float32)
    out = host(L.deform(dev(g), dev(x), res, channels=6))
    ref = C.cayley(cell[:3, None].astype(np.float64))[0] @ x.astype(np.float64) + \
        cell[3:, None].astype(np.float64)
    assert np.max(np.abs(out - ref)) <= 2e-6 * (1.0 + np.max(np.abs(ref)))


@pytest.mark.parametrize("res,n,seed", CASES)
def test_grid_adjoint6_matches_oracle(res, n, seed):
    require_gpu()
    g, x = _inputs(res, n, seed)
    gout = np.random.default_rng(seed + 100).normal(size=(3, n)).astype(np.float32)
    print(f"grid adjoint6 res={res} n={n}", flush=True)
    gg, _ = L.deform_backward(dev(g), dev(x), dev(gout), res, need_x=False, channels=6)
    gg = host(gg)
    ref = C.grid_adjoint6(g, res, x, gout, 1.0 / len(res))
    assert_rel(gg, ref, 1e-5, "six-channel grid adjoint")
    assert np.all(gg[ref == 0.0] == 0.0)            # untouched nodes are exactly zero


@pytest.mark.parametrize("res,n,seed", CASES[:3])
def test_position_adjoint6_matches_oracle(res, n, seed):
    require_gpu()
    g, x = _inputs(res, n, seed)
    gout = np.random.default_rng(seed + 7).normal(size=(3, n)).astype(np.float32)
    gg, gx = L.deform_backward(dev(g), dev(x), dev(gout), res, channels=6)
    gx = host(gx)
    ok = _off_kinks(x, res)
    assert ok.mean() > 0.9
    ref = C.position_adjoint6(g, res, x, gout, 1.0 / len(res))
    # compare the part that goes through the grid (R^T gout taken out of both)
    z = C.transform(g, res, x, 1.0 / len(res))[:3]
    base = np.einsum("nij,in->jn", C.cayley(z), gout.astype(np.float64))
    assert_rel(gx[:, ok] - base[:, ok], ref[:, ok] - base[:, ok], 1e-5, "six-channel position adjoint")
    # ggrids computed in the same call as gx is the same as alone
    gg2, _ = L.deform_backward(dev(g), dev(x), dev(gout), res, need_x=False, channels=6)
    assert torch.equal(gg, gg2)


def test_backward6_bitwise_deterministic_and_empty():
    require_gpu()
    res = (3, 5, 7)
    g, x = _inputs(res, 20_000, 9)
    x[:, :5000] = x[:, :1][:, [0] * 5000] + np.float32(1e-4) * x[:, :5000]   # long runs
    gout = np.random.default_rng(1).normal(size=(3, 20_000)).astype(np.float32)
    a = L.deform_backward(dev(g), dev(x), dev(gout), res, channels=6)
    b = L.deform_backward(dev(g), dev(x), dev(gout), res, channels=6)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    e = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    gg, gx = L.deform_backward(dev(g), e, e, res, channels=6)
    assert torch.count_nonzero(gg).item() == 0 and gx.shape == (3, 0)
    assert L.deform(dev(g), e, res, channels=6).shape == (3, 0)


def test_paper_schedule_200k_points_sampled():
    """The paper's grid (L = 10, R = 2l - 1, six channels) at 200,000 points in
    [-1, 1]^3: the warp on a sample of points, the grid adjoint on every node."""
    require_gpu()
    res = PAPER_RES
    n = 200_000
    g, x = _inputs(res, n, 11, lim=1.0)
    gout = np.random.default_rng(12).normal(size=(3, n)).astype(np.float32)
    out = host(L.deform(dev(g), dev(x), res, channels=6))
    idx = np.random.default_rng(13).choice(n, 3000, replace=False)
    ref = C.warp6(g, res, x[:, idx], 0.1)
    assert np.max(np.abs(out[:, idx] - ref) / (1.0 + np.abs(ref))) <= 4e-6
    gg, _ = L.deform_backward(dev(g), dev(x), dev(gout), res, need_x=False, channels=6)
    assert_rel(host(gg), C.grid_adjoint6(g, res, x, gout, 0.1), 1e-5, "grid adjoint, L = 10")
