"""Pins for the oracle's robust Chamfer distance (Sec. 3.4, Eq. 11-13)."""
import json
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import chamfer as C

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_alpha_matches_paper():
    assert C.ALPHA == json.load(open(GOLD))["alpha"]["value"]


def test_identical_clouds_zero_and_identity_nn():
    rng = np.random.default_rng(0)
    p = rng.uniform(-1, 1, (3, 300)).astype(np.float32)
    lab, lba, na, nb = C.chamfer(p, p)
    assert lab == 0.0 and lba == 0.0
    assert np.array_equal(na, np.arange(300)) and np.array_equal(nb, np.arange(300))


def test_symmetry():
    rng = np.random.default_rng(1)
    a = rng.uniform(-1, 1, (3, 200)).astype(np.float32)
    b = rng.uniform(-1, 1, (3, 150)).astype(np.float32)
    l1 = C.chamfer(a, b)
    l2 = C.chamfer(b, a)
    assert l1[0] == l2[1] and l1[1] == l2[0]


def test_alpha_zero_is_plain_chamfer_kdtree():
    # library cross-check: scipy's k-d tree in float64, compared by distance
    rng = np.random.default_rng(2)
    a = rng.uniform(-1, 1, (3, 2000)).astype(np.float32)
    b = rng.uniform(-1, 1, (3, 1500)).astype(np.float32)
    lab, lba, na, nb = C.chamfer(a, b, alpha=0.0)
    da, _ = cKDTree(b.T.astype(np.float64)).query(a.T.astype(np.float64))
    db, _ = cKDTree(a.T.astype(np.float64)).query(b.T.astype(np.float64))
    assert abs(lab - np.mean(da ** 2)) <= 1e-6 * lab
    assert abs(lba - np.mean(db ** 2)) <= 1e-6 * lba
    # each float32-contract neighbour is a true nearest neighbour up to the
    # float32 rounding of the squared distance
    s = C.sqdist(a, b, na)
    assert np.all(s <= da ** 2 * (1 + 4e-7) + 1e-12)


def _loops(a, b, alpha):
    n, m = a.shape[1], b.shape[1]
    nn = []
    tot = 0.0
    for i in range(n):
        best, bj = None, -1
        for j in range(m):
            dx = np.float32(a[0, i] - b[0, j])
            dy = np.float32(a[1, i] - b[1, j])
            dz = np.float32(a[2, i] - b[2, j])
            d = np.float32(np.float32(np.float32(dx * dx) + np.float32(dy * dy)) + np.float32(dz * dz))
            if best is None or d < best:
                best, bj = d, j
        nn.append(bj)
        s = sum((float(a[k, i]) - float(b[k, bj])) ** 2 for k in range(3))
        tot += np.exp(-alpha * s) * s
    return np.array(nn), tot / n


def test_tiny_brute_force_loops_with_ties():
    rng = np.random.default_rng(3)
    a = rng.uniform(-1, 1, (3, 23)).astype(np.float32)
    b = rng.uniform(-1, 1, (3, 31)).astype(np.float32)
    b[:, 20] = b[:, 5]          # exact duplicate: the lower index must win
    b[:, 30] = b[:, 7]
    a[:, 3] = b[:, 5]
    a[:, 4] = b[:, 7]
    na, la = _loops(a, b, 5.56)
    nb, lb = _loops(b, a, 5.56)
    lab, lba, na2, nb2 = C.chamfer(a, b)
    assert np.array_equal(na, na2) and np.array_equal(nb, nb2)
    assert na2[3] == 5 and na2[4] == 7
    assert abs(lab - la) <= 1e-15 and abs(lba - lb) <= 1e-15


def test_fp32_contract_vs_fp64_only_near_ties():
    rng = np.random.default_rng(4)
    a = rng.uniform(-1, 1, (3, 3000)).astype(np.float32)
    b = (a + rng.normal(0, 0.01, a.shape)).astype(np.float32)
    n32 = C.nn_fp32(a, b)
    n64 = C.nn_fp64(a, b)
    diff = n32 != n64
    s32 = C.sqdist(a, b, n32)
    s64 = C.sqdist(a, b, n64)
    assert np.all(s64 <= s32)
    assert np.all(s32[diff] - s64[diff] <= 4e-7 * s64[diff] + 1e-12)


@pytest.mark.parametrize("alpha", [0.0, 5.56])
def test_gradient_finite_difference_frozen_assignment(alpha):
    rng = np.random.default_rng(5)
    a = rng.uniform(-1, 1, (3, 40))
    b = rng.uniform(-1, 1, (3, 50))
    na = C.nn_fp64(a, b)
    nb = C.nn_fp64(b, a)
    wab, wba = 0.7, 1.3

    def loss(x):
        return wab * C.direction_loss(x, b, na, alpha) + wba * C.direction_loss(b, x, nb, alpha)

    g = C.gradient(a, b, na, nb, alpha, wab, wba)
    h = 1e-6
    for i in range(0, 40, 3):
        for c in range(3):
            ap, am = a.copy(), a.copy()
            ap[c, i] += h
            am[c, i] -= h
            fd = (loss(ap) - loss(am)) / (2 * h)
            assert abs(fd - g[c, i]) <= 1e-7 * max(1.0, abs(g[c, i]))


def test_empty_set_rejected():
    with pytest.raises(ValueError):
        C.nn_fp32(np.zeros((3, 0), np.float32), np.zeros((3, 4), np.float32))
