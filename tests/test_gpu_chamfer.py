"""GPU parity of pdg_chamfer against the oracle (Eq. 11-13): indices
bit-exact under the float32 contract, losses and gradients to 1e-5."""
import numpy as np
import pytest
import torch

import synth
from oracle import chamfer as C
from paper_2509_18097_amd import _lib as L
from _gpu import assert_rel, dev, host, require_gpu

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (1, 700), (700, 1), (1000, 1537), (4096, 4096), (5000, 2562)]


def _clouds(n, m, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    b = rng.uniform(-1, 1, (3, m)).astype(np.float32)
    return a, b


MODES = ["fp32", "bf16", "fp32cull"]


@pytest.mark.parametrize("n,m", SIZES)
@pytest.mark.parametrize("mode", MODES)
def test_indices_and_losses(n, m, mode):
    require_gpu()
    a, b = _clouds(n, m, n * 7 + m)
    print(f"chamfer {mode} n={n} m={m}", flush=True)
    loss, na, nb, _ = L.chamfer(dev(a), dev(b), mode=mode)
    na, nb, loss = host(na), host(nb), host(loss)
    ra = C.nn_fp32(a, b)
    rb = C.nn_fp32(b, a)
    assert np.array_equal(na, ra)
    assert np.array_equal(nb, rb)
    la = C.direction_loss(a, b, ra)
    lb = C.direction_loss(b, a, rb)
    assert abs(loss[0] - la) <= 1e-10 * abs(la) + 1e-300
    assert abs(loss[1] - lb) <= 1e-10 * abs(lb) + 1e-300


@pytest.mark.parametrize("mode", MODES)
def test_ties_go_to_lowest_index(mode):
    require_gpu()
    a, b = _clouds(3000, 2000, 3)
    b[:, 1500:] = b[:, :500]           # exact duplicates at higher indices
    a[:, :200] = b[:, 1700:1900]       # queries sitting exactly on duplicates
    loss, na, nb, _ = L.chamfer(dev(a), dev(b), mode=mode)
    na = host(na)
    assert np.array_equal(na, C.nn_fp32(a, b))
    assert np.all(na[:200] == np.arange(200, 400))
    assert np.array_equal(host(nb), C.nn_fp32(b, a))


@pytest.mark.parametrize("mode", MODES)
def test_identical_clouds_zero(mode):
    require_gpu()
    a, _ = _clouds(2048, 1, 4)
    loss, na, nb, ga = L.chamfer(dev(a), dev(a), mode=mode, need_grad=True)
    assert np.all(host(loss) == 0.0)
    assert np.array_equal(host(na), np.arange(2048)) and np.array_equal(host(nb), np.arange(2048))
    assert np.all(host(ga) == 0.0)


@pytest.mark.parametrize("alpha", [0.0, 5.56])
def test_gradient_matches_oracle(alpha):
    require_gpu()
    a, b = _clouds(3000, 4500, 5)
    w = np.array([0.3, 1.7])
    loss, na, nb, ga = L.chamfer(dev(a), dev(b), alpha=alpha, dir_weight=dev(w), need_grad=True)
    na, nb = host(na), host(nb)
    ref = C.gradient(a, b, na, nb, alpha, w[0], w[1])
    assert_rel(host(ga), ref, 1e-5, "chamfer gradient")


@pytest.mark.parametrize("mode", MODES)
def test_precision_pair_200k_sampled(mode):
    """200k x 200k cloud pair (uniform cube, jitter 0.01): indices checked on a
    random sample of queries against the brute-force oracle, losses checked
    from the returned assignment."""
    require_gpu()
    p, q = synth.cloud_pair_cube(seed=0, n=200_000)
    print(f"chamfer 200k x 200k {mode}", flush=True)
    loss, na, nb, _ = L.chamfer(dev(p), dev(q), mode=mode)
    na, nb, loss = host(na), host(nb), host(loss)
    rng = np.random.default_rng(0)
    for qs, cs, nn in ((p, q, na), (q, p, nb)):
        idx = rng.choice(qs.shape[1], 400, replace=False)
        ref = C.nn_fp32(qs[:, idx], cs, workers=8)
        assert np.array_equal(nn[idx], ref)
    assert abs(loss[0] - C.direction_loss(p, q, na)) <= 1e-10 * loss[0]
    assert abs(loss[1] - C.direction_loss(q, p, nb)) <= 1e-10 * loss[1]


@pytest.mark.parametrize("mode", ["bf16", "fp32cull"])
def test_screen_equals_exact_everywhere_200k(mode):
    """The screened and the culled searches return exactly the exact search's
    indices on every query of the 200k x 200k pair (both directions)."""
    require_gpu()
    p, q = synth.cloud_pair_cube(seed=1, n=200_000)
    l0, a0, b0, _ = L.chamfer(dev(p), dev(q), mode="fp32")
    l1, a1, b1, _ = L.chamfer(dev(p), dev(q), mode=mode)
    assert torch.equal(a0, a1) and torch.equal(b0, b1)
    assert torch.equal(l0, l1)


@pytest.mark.parametrize("mode", ["bf16", "fp32cull"])
def test_screen_far_and_clustered_points(mode):
    """Coordinates far from the origin (large |x| widens the screen bound) and
    many near-duplicates (narrow gaps) still give the exact indices."""
    require_gpu()
    rng = np.random.default_rng(9)
    base = rng.uniform(-1, 1, (3, 64))
    a = (np.repeat(base, 40, axis=1) + rng.normal(0, 1e-4, (3, 2560)) + 3.0).astype(np.float32)
    b = (np.repeat(base, 30, axis=1) + rng.normal(0, 1e-4, (3, 1920)) + 3.0).astype(np.float32)
    _, na, nb, _ = L.chamfer(dev(a), dev(b), mode=mode)
    assert np.array_equal(host(na), C.nn_fp32(a, b))
    assert np.array_equal(host(nb), C.nn_fp32(b, a))
