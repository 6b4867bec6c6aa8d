"""Grid Sobolev preconditioner (paper Sec. 3.2, Eq. 3) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 3 replaces the gradient of level l by (I + lambda L^l)^{-2} times it,
where L^l is the Laplacian of the adjacency between neighbouring grid cells.

Readings:
* L = D - A is the combinatorial graph Laplacian of the 6-face-neighbour
  graph of the R^3 box of cells, unscaled by the cell size; cells on the box
  boundary simply have fewer neighbours (free / Neumann boundary).
* The three channels, the levels and the transitions are independent systems.

Two independent ways of applying (I + lambda L)^{-2} are given:
* ``apply_dense``  -- build I + lambda L explicitly, Cholesky-factor it and
  solve twice (small boxes only).
* ``apply_dct``    -- the closed form.  The orthonormal DCT-II basis
  diagonalises the Laplacian of a path with free ends (eigenvalues
  2 - 2 cos(pi k / n)); the box Laplacian is the Kronecker sum of three path
  Laplacians, so (I + lambda L)^{-2} is diagonal in the separable 3-D DCT-II
  basis with entries (1 + lambda (mu_i + mu_j + mu_k))^{-2}.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def laplacian(r: int) -> sp.csr_matrix:
    """Combinatorial 6-neighbour Laplacian of an r^3 cell box, flat index
    (z*r + y)*r + x, built edge by edge."""
    n = r ** 3
    ids = np.arange(n).reshape(r, r, r)          # [z, y, x]
    rows, cols = [], []
    for axis in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, r - 1)
        hi[axis] = slice(1, r)
        a = ids[tuple(lo)].reshape(-1)
        b = ids[tuple(hi)].reshape(-1)
        rows += [a, b]
        cols += [b, a]
    if rows:
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
    else:
        rows = cols = np.zeros(0, np.int64)
    adj = sp.csr_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(n, n))
    deg = np.asarray(adj.sum(axis=1)).reshape(-1)
    return (sp.diags(deg) - adj).tocsr()


def apply_dense(g: np.ndarray, r: int, lam: float) -> np.ndarray:
    """(I + lam L)^{-2} g via a dense Cholesky factorisation.  g: (..., r^3)."""
    a = np.eye(r ** 3) + lam * laplacian(r).toarray()
    fac = sla.cho_factor(a)
    g = np.asarray(g, dtype=np.float64)
    flat = g.reshape(-1, r ** 3).T
    y = sla.cho_solve(fac, flat)
    x = sla.cho_solve(fac, y)
    return x.T.reshape(g.shape)


def dct_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix C[k, i] = s_k cos(pi k (i + 1/2) / n)."""
    k = np.arange(n)[:, None]
    i = np.arange(n)[None, :]
    c = np.cos(np.pi * k * (i + 0.5) / n) * np.sqrt(2.0 / n)
    c[0, :] = np.sqrt(1.0 / n)
    return c


def apply_dct(g: np.ndarray, r: int, lam: float) -> np.ndarray:
    """(I + lam L)^{-2} g by the separable DCT-II closed form.  g: (..., r^3)."""
    g = np.asarray(g, dtype=np.float64)
    c = dct_matrix(r)
    mu = 2.0 - 2.0 * np.cos(np.pi * np.arange(r) / r)
    scale = (1.0 + lam * (mu[:, None, None] + mu[None, :, None] + mu[None, None, :])) ** -2
    out = np.empty(g.reshape(-1, r ** 3).shape)
    for b, v in enumerate(g.reshape(-1, r, r, r)):              # [z, y, x]
        h = np.einsum("az,zyx->ayx", c, v)
        h = np.einsum("by,ayx->abx", c, h)
        h = np.einsum("cx,abx->abc", c, h)
        h *= scale
        h = np.einsum("cx,abc->abx", c, h)
        h = np.einsum("by,abx->ayx", c, h)
        h = np.einsum("az,ayx->zyx", c, h)
        out[b] = h.reshape(-1)
    return out.reshape(g.shape)


def apply_levels(flat: np.ndarray, res, lams, method: str = "dct", channels: int = 3) -> np.ndarray:
    """Precondition one transition's packed gradient level by level (Eq. 3),
    every channel of a level alike."""
    fn = apply_dct if method == "dct" else apply_dense
    out, off = [], 0
    flat = np.asarray(flat, dtype=np.float64)
    for r, lam in zip(res, lams):
        n = channels * r ** 3
        out.append(fn(flat[off:off + n].reshape(channels, r ** 3), r, lam).reshape(-1))
        off += n
    return np.concatenate(out)


def cg_iterations(lam: float, tol: float = 1e-7) -> int:
    """A-priori conjugate-gradient iteration count for I + lam L.

    Every eigenvalue of the box Laplacian lies in [0, 12), so the condition
    number is below kappa = 1 + 12 lam and the textbook bound
    2 ((sqrt k - 1)/(sqrt k + 1))^i <= tol gives the count.
    """
    kappa = 1.0 + 12.0 * lam
    rho = (np.sqrt(kappa) - 1.0) / (np.sqrt(kappa) + 1.0)
    if rho <= 0.0:
        return 1
    return int(np.ceil(np.log(2.0 / tol) / -np.log(rho)))
