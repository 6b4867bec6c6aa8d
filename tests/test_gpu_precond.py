"""GPU parity of pdg_precondition (CG) against the oracle's exact
(I + lambda L)^-2 (Eq. 3), plus its invariants."""
import numpy as np
import pytest

from oracle import precond as P
from paper_2509_18097_amd import _lib as L
from _gpu import assert_rel, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def _lams(k):
    return [0.25 * 1.5 ** l for l in range(k)]


@pytest.mark.parametrize("method", ["cg", "dct"])
@pytest.mark.parametrize("res,batch", [((1, 2, 3, 5), 2), ((8, 16, 32), 1), ((16, 32, 64), 1),
                                       ((9, 13), 3), ((33, 40), 1)])
def test_matches_exact(res, batch, method):
    require_gpu()
    rng = np.random.default_rng(sum(res) + batch)
    g = rng.normal(size=batch * L.grid_size(res)).astype(np.float32)
    print(f"precondition {method} res={res} batch={batch}", flush=True)
    out = host(L.precondition(dev(g), res, _lams(len(res)), batch=batch, method=method))
    stack = L.grid_size(res)
    ref = np.concatenate([P.apply_levels(g[b * stack:(b + 1) * stack], res, _lams(len(res)))
                          for b in range(batch)])
    off = 0
    for r in res:
        for b in range(batch):
            sl = slice(b * stack + off, b * stack + off + 3 * r ** 3)
            assert_rel(out[sl], ref[sl], 1e-5, f"R={r}")
        off += 3 * r ** 3


@pytest.mark.parametrize("method", ["cg", "dct"])
def test_finest_level_128(method):
    require_gpu()
    res = (128,)
    rng = np.random.default_rng(3)
    g = rng.normal(size=L.grid_size(res)).astype(np.float32)
    lam = [0.84375]
    out = host(L.precondition(dev(g), res, lam, method=method))
    ref = P.apply_levels(g, res, lam)
    assert_rel(out, ref, 1e-5, "R=128")


def test_dct_level_256():
    """The finest level of the 5-level differentiation stack (256^3)."""
    require_gpu()
    res = (256,)
    rng = np.random.default_rng(7)
    g = rng.normal(size=L.grid_size(res)).astype(np.float32)
    lam = [1.265625]
    out = host(L.precondition(dev(g), res, lam, method="dct"))
    # oracle on one channel (the three are independent systems)
    n = 256 ** 3
    ref = P.apply_dct(g[:n].astype(np.float64), 256, lam[0])
    assert_rel(out[:n], ref, 1e-5, "R=256")


def test_dct_matches_cg_on_step_levels():
    require_gpu()
    res = (16, 32, 64, 128)
    rng = np.random.default_rng(8)
    g = rng.normal(size=2 * L.grid_size(res)).astype(np.float32)
    a = host(L.precondition(dev(g), res, _lams(4), batch=2, method="cg"))
    b = host(L.precondition(dev(g), res, _lams(4), batch=2, method="dct"))
    assert_rel(b, a, 1e-5, "dct vs cg")


@pytest.mark.parametrize("method", ["cg", "dct"])
def test_invariants_on_gpu(method):
    require_gpu()
    res = (6, 12)
    rng = np.random.default_rng(4)
    g = rng.normal(size=L.grid_size(res)).astype(np.float32)
    out = host(L.precondition(dev(g), res, [0.5, 1.0], method=method))
    off = 0
    for r in res:
        for c in range(3):
            sl = slice(off + c * r ** 3, off + (c + 1) * r ** 3)
            assert abs(out[sl].astype(np.float64).sum() - g[sl].astype(np.float64).sum()) <= \
                1e-5 * np.abs(g[sl]).sum()
        off += 3 * r ** 3
    const = np.full(L.grid_size(res), 0.375, np.float32)
    out = host(L.precondition(dev(const), res, [0.5, 1.0], method=method))
    assert np.max(np.abs(out - 0.375)) <= 1e-6
    # lambda = 0 leaves the gradient untouched
    out = host(L.precondition(dev(g), res, [0.0, 0.0], method=method))
    assert np.array_equal(out, g)


def test_dct_fast_levels_on_misaligned_and_unaligned_layouts():
    """The fast passes (R = 16, 32, 64, 128) read and write float4; a buffer
    that is not 16-byte aligned (a view one float into an allocation) or a level
    offset that is not a multiple of 4 floats (a 3^3 level before it) takes the
    generic passes, with the same result."""
    require_gpu()
    import torch
    for res in ((64,), (3, 64)):
        rng = np.random.default_rng(11 + len(res))
        g = rng.normal(size=L.grid_size(res)).astype(np.float32)
        lam = _lams(len(res))
        ref = P.apply_levels(g, res, lam)
        aligned = host(L.precondition(dev(g), res, lam, method="dct"))
        buf = torch.zeros(g.size + 1, dtype=torch.float32, device="cuda")
        buf[1:] = dev(g)
        shifted = host(L.precondition(buf[1:], res, lam, method="dct"))
        for out, what in ((aligned, "aligned"), (shifted, "shifted")):
            off = 0
            for r in res:
                sl = slice(off, off + 3 * r ** 3)
                assert_rel(out[sl], ref[sl], 1e-5, f"{what} res={res} R={r}")
                off += 3 * r ** 3
