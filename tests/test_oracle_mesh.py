"""Pins for the oracle's mesh preconditioner (Sec. 3.2, 3.6): the cycle graph's
Laplacian has the known Fourier spectrum, so (I + lam L)^{-2} of a Fourier mode
is the mode divided by (1 + lam (2 - 2 cos(2 pi k / n)))^2; constants pass
unchanged; lam = 0 is the identity; the operator is symmetric; a grid graph's
Laplacian has the degrees of a grid."""
import numpy as np

from oracle import mesh as M


def _cycle(n):
    i = np.arange(n)
    return np.stack([i, (i + 1) % n])


def test_cycle_fourier_modes():
    n, lam = 40, 16.0
    for k in (0, 1, 5, 20):
        mode = np.cos(2 * np.pi * k * np.arange(n) / n)
        g = np.stack([mode, 2 * mode, -mode])
        mu = 2.0 - 2.0 * np.cos(2 * np.pi * k / n)
        out = M.precondition(n, _cycle(n), lam, g)
        np.testing.assert_allclose(out, g / (1.0 + lam * mu) ** 2, atol=1e-12)


def test_constants_identity_and_symmetry():
    rng = np.random.default_rng(0)
    v = 60
    e = np.unique(np.sort(rng.integers(0, v, (2, 200)), axis=0), axis=1)
    e = e[:, e[0] != e[1]]
    ones = np.ones((3, v))
    np.testing.assert_allclose(M.precondition(v, e, 16.0, ones), ones, atol=1e-12)
    g = rng.normal(size=(3, v))
    np.testing.assert_allclose(M.precondition(v, e, 0.0, g), g, atol=1e-14)
    a, b = rng.normal(size=(1, v)), rng.normal(size=(1, v))
    pa, pb = M.precondition(v, e, 5.0, a), M.precondition(v, e, 5.0, b)
    assert abs(np.sum(pa * b) - np.sum(a * pb)) <= 1e-12 * np.sum(np.abs(a * b))


def test_grid_graph_degrees_and_max_degree():
    # a 4 x 3 grid: corner degree 2, border 3, interior 4
    idx = np.arange(12).reshape(3, 4)
    e = np.concatenate([np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()]),
                        np.stack([idx[:-1].ravel(), idx[1:].ravel()])], axis=1)
    lap = M.laplacian(12, e).toarray()
    assert lap.diagonal().tolist() == [2, 3, 3, 2, 3, 4, 4, 3, 2, 3, 3, 2]
    assert np.allclose(lap.sum(axis=1), 0.0)
    assert M.max_degree(12, e) == 4
