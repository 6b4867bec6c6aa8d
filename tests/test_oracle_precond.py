"""Pins for the oracle's grid preconditioner (Sec. 3.2, Eq. 3)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import precond as P


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8])
def test_laplacian_structure(r):
    lap = P.laplacian(r).toarray()
    assert np.allclose(lap, lap.T)
    assert np.allclose(lap.sum(axis=1), 0.0)
    deg = np.diag(lap).reshape(r, r, r)
    # degree = number of face neighbours inside the box
    for z in range(r):
        for y in range(r):
            for x in range(r):
                want = sum((c > 0) + (c < r - 1) for c in (x, y, z))
                assert deg[z, y, x] == want
    ev = np.linalg.eigvalsh(lap)
    assert ev.min() > -1e-12 and ev.max() < 12.0


def test_dct_diagonalises_path_laplacian():
    # textbook fact: the orthonormal DCT-II basis diagonalises the free-end path
    # Laplacian with eigenvalues 2 - 2 cos(pi k / n)
    for n in (2, 5, 16):
        lp = P.laplacian(n).toarray()
        # the path along x is the sub-block for y = z = 0 when restricted: build directly
        path = np.diag(np.r_[1.0, 2.0 * np.ones(n - 2), 1.0] if n > 1 else [0.0]) \
            - np.eye(n, k=1) - np.eye(n, k=-1)
        c = P.dct_matrix(n)
        assert np.allclose(c @ c.T, np.eye(n), atol=1e-14)
        mu = 2 - 2 * np.cos(np.pi * np.arange(n) / n)
        np.testing.assert_allclose(c @ path @ c.T, np.diag(mu), atol=1e-13)
        assert lp.shape == (n ** 3, n ** 3)


@pytest.mark.parametrize("r,lam", [(2, 0.25), (4, 0.375), (6, 0.4), (9, 1.265625)])
def test_dense_cholesky_equals_dct(r, lam):
    rng = np.random.default_rng(r)
    g = rng.normal(size=(3, r ** 3))
    a = P.apply_dense(g, r, lam)
    b = P.apply_dct(g, r, lam)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("method", ["dense", "dct"])
def test_invariants(method):
    r, lam = 5, 0.8
    fn = P.apply_dense if method == "dense" else P.apply_dct
    rng = np.random.default_rng(11)
    g = rng.normal(size=r ** 3)
    out = fn(g, r, lam)
    # 1^T (I + lam L)^{-1} = 1^T because L 1 = 0: the sum is conserved
    assert abs(out.sum() - g.sum()) <= 1e-12 * np.abs(g).sum()
    # a constant gradient is returned unchanged
    np.testing.assert_allclose(fn(np.full(r ** 3, 0.37), r, lam), 0.37, rtol=0, atol=1e-14)
    # lam = 0 is the identity
    np.testing.assert_allclose(fn(g, r, 0.0), g, rtol=0, atol=1e-13)
    # symmetric operator
    h = rng.normal(size=r ** 3)
    assert abs(np.dot(fn(g, r, lam), h) - np.dot(g, fn(h, r, lam))) <= 1e-12
    # smoothing: the Laplacian energy of the output is below that of the input
    lap = P.laplacian(r)
    assert out @ (lap @ out) < g @ (lap @ g)


def test_equals_sparse_direct_solve_twice():
    r, lam = 12, 0.5625
    rng = np.random.default_rng(3)
    g = rng.normal(size=r ** 3)
    import scipy.sparse as sp
    a = (sp.identity(r ** 3) + lam * P.laplacian(r)).tocsc()
    lu = spla.splu(a)
    ref = lu.solve(lu.solve(g))
    np.testing.assert_allclose(P.apply_dct(g, r, lam), ref, rtol=0, atol=1e-12)


def test_levels_packed_independently():
    res, lams = (2, 3), (0.25, 0.375)
    rng = np.random.default_rng(4)
    flat = rng.normal(size=3 * (8 + 27))
    out = P.apply_levels(flat, res, lams)
    np.testing.assert_allclose(out[:24], P.apply_dense(flat[:24].reshape(3, 8), 2, 0.25).reshape(-1), atol=1e-13)
    np.testing.assert_allclose(out[24:], P.apply_dense(flat[24:].reshape(3, 27), 3, 0.375).reshape(-1), atol=1e-13)


@pytest.mark.parametrize("lam", [0.25, 0.84375, 1.265625])
def test_cg_count_reaches_tolerance(lam):
    # the a-priori count from kappa = 1 + 12 lam is enough for a textbook CG
    import scipy.sparse as sp
    r = 10
    k = P.cg_iterations(lam, 1e-7)
    a = (sp.identity(r ** 3) + lam * P.laplacian(r)).tocsr()
    rng = np.random.default_rng(5)
    b = rng.normal(size=r ** 3)
    x = np.zeros_like(b)
    res = b.copy()
    p = res.copy()
    rr = res @ res
    for _ in range(k):
        ap = a @ p
        al = rr / (p @ ap)
        x += al * p
        res -= al * ap
        rn = res @ res
        p = res + (rn / rr) * p
        rr = rn
    exact = spla.spsolve(a.tocsc(), b)
    e = x - exact
    assert np.sqrt(e @ (a @ e)) <= 1e-7 * np.sqrt(exact @ (a @ exact)) * 2
    # and the bound is not vacuous: half the iterations do not reach it
    assert k >= 10
