"""Mesh-vertex preconditioner (paper Sec. 3.2 and Sec. 3.6) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper preconditions the updates of the initial mesh's vertices X_0 the way
it preconditions the grids (Eq. 3), with the mesh Laplacian and a smoothness
weight lambda = 16 (Sec. 3.6, after Nicolet et al.):

    g  ->  (I + lambda L)^{-2} g,      L = D - A of the mesh's edge graph,

applied to each coordinate channel.  Together with L_mesh = CD_R(X_0, P_0)
(Eq. 10, the robust Chamfer of ``chamfer``) this is the template side of the
optimisation.

Readings (the paper does not state them):
* L is the combinatorial Laplacian of the undirected edge graph, built from
  the given edge list with each listed edge counted once (a list holding both
  (a, b) and (b, a) describes a double edge); unweighted, no cotangent terms.
* The update rule around the preconditioned gradient (Adam or plain descent,
  learning rate 1e-4) is the caller's.

Here both solves are sparse LU factorisations in float64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian(v: int, edges: np.ndarray) -> sp.csr_matrix:
    """L = D - A (v x v) of the edge list edges (2, E)."""
    e = np.asarray(edges, dtype=np.int64)
    a = sp.coo_matrix((np.ones(e.shape[1]), (e[0], e[1])), shape=(v, v))
    a = (a + a.T).tocsr()
    deg = np.asarray(a.sum(axis=1)).ravel()
    return (sp.diags(deg) - a).tocsr()


def precondition(v: int, edges: np.ndarray, lam: float, g: np.ndarray) -> np.ndarray:
    """(I + lam L)^{-2} g for g (3, v), two sparse solves per channel: (3, v) float64."""
    m = (sp.identity(v) + lam * laplacian(v, edges)).tocsc()
    lu = spla.splu(m)
    g = np.asarray(g, dtype=np.float64)
    return np.stack([lu.solve(lu.solve(g[c])) for c in range(g.shape[0])])


def max_degree(v: int, edges: np.ndarray) -> int:
    e = np.asarray(edges, dtype=np.int64)
    return int(np.bincount(e.reshape(-1), minlength=v).max()) if e.size else 0
