"""Pins for the oracle's trilinear warp (Sec. 3.1, Eq. 1) and its adjoints.

Each test checks the oracle against something other than itself: exact
identities of trilinear interpolation, an independent hat-function
formulation written with explicit loops, and finite differences.
"""
import itertools

import numpy as np
import pytest

from oracle import warp as W


def _rand_grid(rng, res, scale=1.0):
    return rng.normal(0.0, scale, 3 * sum(r ** 3 for r in res))


def test_zero_grid_is_identity_bitwise():
    rng = np.random.default_rng(1)
    x = rng.uniform(-1.2, 1.2, (3, 500)).astype(np.float32)
    res = (1, 2, 5, 8)
    out = W.warp(np.zeros(3 * sum(r ** 3 for r in res)), res, x, 0.25)
    assert np.array_equal(out, x.astype(np.float64))


def test_constant_grid_is_translation():
    # weights sum to one on every level and levels are averaged (Eq. 1), so a
    # constant c in every cell of every level moves every point by exactly c,
    # also outside the cube (border clamp).
    rng = np.random.default_rng(2)
    x = rng.uniform(-1.3, 1.3, (3, 400))
    res = (1, 3, 4, 16)
    c = np.array([0.3, -0.2, 0.05])
    flat = np.concatenate([np.repeat(c, r ** 3) for r in res])
    out = W.warp(flat, res, x, 1.0 / len(res))
    np.testing.assert_allclose(out - x, np.repeat(c[:, None], x.shape[1], 1), rtol=0, atol=1e-14)


def test_affine_field_reproduced_inside_hull():
    # trilinear interpolation is exact on affine functions: a grid sampled at
    # the cell centres -1 + (2i+1)/R from g(x) = Bx + b reproduces g inside the
    # hull of the centres of every level.
    rng = np.random.default_rng(3)
    bm = rng.normal(size=(3, 3))
    bv = rng.normal(size=3)
    res = (2, 4, 7)
    levels = []
    for r in res:
        cen = -1.0 + (2.0 * np.arange(r) + 1.0) / r
        z, y, xx = np.meshgrid(cen, cen, cen, indexing="ij")
        pts = np.stack([xx.ravel(), y.ravel(), z.ravel()])
        levels.append((bm @ pts + bv[:, None]).reshape(3, r, r, r))
    flat = W.pack(levels)
    lim = 1.0 - 1.0 / min(res)
    x = rng.uniform(-lim, lim, (3, 300))
    out = W.warp(flat, res, x, 1.0 / len(res))
    np.testing.assert_allclose(out - x, bm @ x + bv[:, None], rtol=0, atol=1e-12)


def _hat_interp(g, r, p):
    """Independent formulation: sum over all nodes of the tensor-product hat
    function max(0, 1 - |u - i|) with u clamped to the hull of the centres."""
    if r == 1:
        return g[:, 0, 0, 0].copy()
    u = [min(max((p[a] + 1.0) * r / 2.0 - 0.5, 0.0), r - 1.0) for a in range(3)]
    val = np.zeros(3)
    for k, j, i in itertools.product(range(r), repeat=3):
        w = max(0.0, 1 - abs(u[0] - i)) * max(0.0, 1 - abs(u[1] - j)) * max(0.0, 1 - abs(u[2] - k))
        if w:
            val += w * g[:, k, j, i]
    return val


@pytest.mark.parametrize("res", [(2,), (3,), (1, 2, 3)])
def test_brute_force_hat_functions(res):
    rng = np.random.default_rng(4)
    flat = _rand_grid(rng, res)
    levels = W.unpack(flat, res)
    x = rng.uniform(-1.2, 1.2, (3, 60))
    x[:, 0] = [-1.0, 1.0, 0.0]                  # exact border / centre values
    out = W.warp(flat, res, x, 1.0 / len(res))
    for n in range(x.shape[1]):
        ref = sum(_hat_interp(g, r, x[:, n]) for g, r in zip(levels, res)) / len(res)
        np.testing.assert_allclose(out[:, n] - x[:, n], ref, rtol=0, atol=1e-13)


def test_grid_adjoint_dot_product():
    # the warp is linear in G, so <A G, gbar> = <G, A^T gbar> to rounding
    rng = np.random.default_rng(5)
    res = (1, 4, 9)
    x = rng.uniform(-1.1, 1.1, (3, 700))
    g = _rand_grid(rng, res)
    gbar = rng.normal(size=(3, 700))
    lhs = np.sum((W.warp(g, res, x, 1 / 3) - x) * gbar)
    rhs = np.dot(g, W.grid_adjoint(res, x, gbar, 1 / 3))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_grid_adjoint_finite_difference():
    rng = np.random.default_rng(6)
    res = (2, 3)
    x = rng.uniform(-1, 1, (3, 40))
    g = _rand_grid(rng, res)
    gbar = rng.normal(size=(3, 40))
    grad = W.grid_adjoint(res, x, gbar, 0.5)
    h = 1e-3
    for k in rng.choice(g.size, 12, replace=False):
        gp, gm = g.copy(), g.copy()
        gp[k] += h
        gm[k] -= h
        fd = (np.sum(W.warp(gp, res, x, 0.5) * gbar) - np.sum(W.warp(gm, res, x, 0.5) * gbar)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-9 * max(1.0, abs(fd))


def test_position_adjoint_finite_difference():
    rng = np.random.default_rng(7)
    res = (1, 4, 8)
    g = _rand_grid(rng, res, 0.1)
    x = rng.uniform(-1.2, 1.2, (3, 200))
    # keep samples h away from cell-centre planes and clamp boundaries (kinks)
    h = 1e-6
    ok = np.ones(x.shape[1], bool)
    for r in res[1:]:
        u = (x + 1.0) * r / 2.0 - 0.5
        ok &= np.all(np.abs(u - np.round(u)) > 1e-3, axis=0)
    x = x[:, ok]
    gbar = rng.normal(size=x.shape)
    gx = W.position_adjoint(g, res, x, gbar, 1 / 3)
    for a in range(3):
        xp, xm = x.copy(), x.copy()
        xp[a] += h
        xm[a] -= h
        fd = np.sum((W.warp(g, res, xp, 1 / 3) - W.warp(g, res, xm, 1 / 3)) * gbar, axis=0) / (2 * h)
        np.testing.assert_allclose(gx[a], fd, rtol=1e-6, atol=1e-7)


def test_position_jacobian_zero_when_clamped():
    rng = np.random.default_rng(8)
    res = (4,)
    g = _rand_grid(rng, res)
    x = np.array([[1.5, -1.7, 0.1], [0.2, 0.3, 2.0], [-0.1, 0.0, 0.4]])
    gbar = np.ones_like(x)
    gx = W.position_adjoint(g, res, x, gbar, 1.0)
    assert gx[0, 0] == 1.0 and gx[0, 1] == 1.0 and gx[1, 2] == 1.0


def test_unpack_pack_roundtrip_and_layout():
    res = (2, 3)
    flat = np.arange(3 * (8 + 27), dtype=np.float64)
    lv = W.unpack(flat, res)
    assert lv[0].shape == (3, 2, 2, 2) and lv[1].shape == (3, 3, 3, 3)
    # x fastest: element [c, z, y, x] of level 1 sits at 24 + ((c*3 + z)*3 + y)*3 + x
    assert lv[1][2, 1, 0, 2] == 24 + ((2 * 3 + 1) * 3 + 0) * 3 + 2
    assert np.array_equal(W.pack(lv), flat)
