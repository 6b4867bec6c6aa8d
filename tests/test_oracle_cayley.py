"""Pins for the oracle's six-channel cells (Sec. 3.3, Eq. 4-7) and adjoints.

Each test checks the oracle against something other than itself: the
textbook axis-angle form of a rotation (which fixes the signs of Eq. 6 and the
order of the factors in Eq. 5), the closed form of the Cayley map, the
translation warp it must reduce to when z = 0, an exact rigid motion for a
constant grid, and finite differences for both adjoints.
"""
import numpy as np
import pytest

from oracle import cayley as C
from oracle import warp as W


def _rodrigues(axis, theta):
    """Rotation by theta about the unit axis (right-hand rule), textbook form."""
    k = np.array([[0.0, -axis[2], axis[1]], [axis[2], 0.0, -axis[0]], [-axis[1], axis[0], 0.0]])
    return np.eye(3) + np.sin(theta) * k + (1.0 - np.cos(theta)) * (k @ k)


def test_cayley_is_a_rotation():
    rng = np.random.default_rng(0)
    z = rng.normal(0.0, 1.5, (3, 200))
    r = C.cayley(z)
    eye = np.broadcast_to(np.eye(3), r.shape)
    np.testing.assert_allclose(np.transpose(r, (0, 2, 1)) @ r, eye, atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(r), 1.0, atol=1e-12)


def test_cayley_axis_angle():
    # z = tan(theta / 2) * axis rotates by theta about axis: pins the sign of
    # the skew matrix and the order of the two factors.
    rng = np.random.default_rng(1)
    for _ in range(50):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        theta = rng.uniform(-3.0, 3.0)
        z = (np.tan(theta / 2.0) * axis)[:, None]
        np.testing.assert_allclose(C.cayley(z)[0], _rodrigues(axis, theta), atol=1e-12)
    # a quarter turn about z takes e_x to e_y
    r = C.cayley(np.array([[0.0], [0.0], [1.0]]))[0]
    np.testing.assert_allclose(r @ np.array([1.0, 0.0, 0.0]), [0.0, 1.0, 0.0], atol=1e-15)


def test_cayley_closed_form():
    # (I + Z)(I - Z)^{-1} = I + 2 (Z + Z^2) / (1 + |z|^2) for skew Z
    rng = np.random.default_rng(2)
    z = rng.normal(0.0, 2.0, (3, 100))
    zm = C.skew(z)
    closed = np.eye(3)[None] + 2.0 * (zm + zm @ zm) / (1.0 + np.sum(z * z, axis=0))[:, None, None]
    np.testing.assert_allclose(C.cayley(z), closed, atol=1e-12)


def test_zero_rotation_is_the_translation_warp():
    rng = np.random.default_rng(3)
    res = (1, 3, 5, 8)
    x = rng.uniform(-1.2, 1.2, (3, 300))
    t = [rng.normal(0.0, 0.05, (3, r, r, r)) for r in res]
    flat6 = np.concatenate([np.concatenate([np.zeros((3, r, r, r)), g]).reshape(-1)
                            for g, r in zip(t, res)])
    flat3 = W.pack(t)
    np.testing.assert_allclose(C.warp6(flat6, res, x, 0.25), W.warp(flat3, res, x, 0.25),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("res", [(1, 3, 5, 7, 9, 11, 13, 15, 17, 19), (2, 8)])
def test_constant_grid_is_a_rigid_motion(res):
    # the paper's 2l - 1 schedule (L = 10) and a doubling one: a constant cell
    # vector on every level, averaged (Eq. 1), moves every point rigidly
    rng = np.random.default_rng(4)
    x = rng.uniform(-1.3, 1.3, (3, 200))
    axis = np.array([1.0, 2.0, -0.5])
    axis /= np.linalg.norm(axis)
    theta = 0.7
    z = np.tan(theta / 2.0) * axis
    t = np.array([0.1, -0.2, 0.05])
    cell = np.concatenate([z, t])
    flat = np.concatenate([np.repeat(cell, r ** 3) for r in res])
    out = C.warp6(flat, res, x, 1.0 / len(res))
    ref = _rodrigues(axis, theta) @ x + t[:, None]
    np.testing.assert_allclose(out, ref, atol=1e-12)


def _problem(seed, res, n=40):
    rng = np.random.default_rng(seed)
    flat = rng.normal(0.0, 0.2, C.grid_size(res))
    # keep samples off cell-centre planes (one-sided derivatives) and inside the hull
    x = rng.uniform(-0.8, 0.8, (3, n))
    gout = rng.normal(size=(3, n))
    return flat, x, gout


def test_grid_adjoint_matches_finite_differences():
    res = (1, 3, 4)
    flat, x, gout = _problem(5, res)
    g = C.grid_adjoint6(flat, res, x, gout, 1.0 / 3)
    rng = np.random.default_rng(6)
    h = 1e-6
    for i in rng.choice(flat.size, 60, replace=False):
        e = np.zeros_like(flat)
        e[i] = h
        fd = (np.sum(gout * C.warp6(flat + e, res, x, 1.0 / 3)) -
              np.sum(gout * C.warp6(flat - e, res, x, 1.0 / 3))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * (1.0 + abs(g[i])), (i, fd, g[i])


def test_position_adjoint_matches_finite_differences():
    res = (1, 3, 4)
    flat, x, gout = _problem(7, res)
    gx = C.position_adjoint6(flat, res, x, gout, 1.0 / 3)
    h = 1e-6
    for a in range(3):
        e = np.zeros_like(x)
        e[a] = h
        fd = (np.sum(gout * C.warp6(flat, res, x + e, 1.0 / 3), axis=0) -
              np.sum(gout * C.warp6(flat, res, x - e, 1.0 / 3), axis=0)) / (2 * h)
        np.testing.assert_allclose(gx[a], fd, rtol=1e-6, atol=1e-7)


def test_rotation_adjoint_matches_finite_differences():
    # d<g, R(z) x>/dz from the differentiated Eq. 5 against differences of Eq. 5
    rng = np.random.default_rng(8)
    z = rng.normal(0.0, 0.8, (3, 30))
    x = rng.normal(size=(3, 30))
    g = rng.normal(size=(3, 30))
    an = np.einsum("in,nkij,jn->kn", g, C.dcayley(z), x)
    h = 1e-6
    for k in range(3):
        e = np.zeros_like(z)
        e[k] = h
        fp = np.einsum("in,nij,jn->n", g, C.cayley(z + e), x)
        fm = np.einsum("in,nij,jn->n", g, C.cayley(z - e), x)
        np.testing.assert_allclose(an[k], (fp - fm) / (2 * h), rtol=1e-6, atol=1e-8)
