"""Pruned grids (paper Sec. 3.6, implementation details) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper keeps only the grid cells that hold input points or lie within three
cells of such a cell, which removes more than half of the parameters.  With
cell values interpolated as in Eq. 1, a pruned grid is the dense grid with
every value outside the active set S fixed at zero: its parameters are the
values on S, the gradient of the loss is restricted to S, and the Sobolev
preconditioner of Eq. 3 acts on the graph the kept cells form,

    g_S  ->  (I + lambda L_S)^{-2} g_S,    L_S = D_S - A_S,

A_S the adjacency of the 6-neighbour cell graph restricted to S x S and D_S
its degrees (a kept cell next to a pruned one simply has fewer neighbours, the
same free boundary the box has at its faces).  The DCT closed form no longer
applies to such a domain.

Readings (the paper does not state them):
* The cell of a point s along an axis is floor((s + 1) R / 2) clamped to
  0..R-1 (the R cells partition [-1, 1]), decided in float32 as the GPU
  decides it: (s + 1) rounded to float32, times R/2 rounded to float32.
* The three-cell neighbourhood is the cube of cells at most three cells away
  along every axis (Chebyshev distance <= 3).
* The grid G_t of transition t (frame t-1 to frame t) is pruned by the points
  of both frames it connects, P_{t-1} and P_t (``span = 2``); the mask is
  fixed for the whole optimisation (the input points do not move).
* Adam keeps the moments of pruned cells at zero, so their values stay zero.

Here the active set is built from its definition (every occupied cell marks
the cube around it) and both solves are sparse LU factorisations in float64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import precond as _pc

HALO = 3


def cell_index(x: np.ndarray, r: int) -> np.ndarray:
    """Per-axis cell of every column of x (3, n) at resolution r: (3, n) int64."""
    x = np.asarray(x, dtype=np.float32)
    u = (x + np.float32(1.0)) * np.float32(r / 2)          # float32 like the GPU
    return np.clip(np.floor(u.astype(np.float64)), 0, r - 1).astype(np.int64)


def occupied(points, r: int) -> np.ndarray:
    """Boolean [r, r, r] ([z, y, x]) of the cells holding a point of any of
    the point sets in ``points`` (each (3, n))."""
    occ = np.zeros((r, r, r), dtype=bool)
    for p in points:
        i = cell_index(p, r)
        occ[i[2], i[1], i[0]] = True
    return occ


def active_mask(points, r: int, halo: int = HALO) -> np.ndarray:
    """Boolean [r, r, r]: cells within ``halo`` cells (Chebyshev) of an occupied
    cell, each occupied cell marking the cube around it."""
    occ = occupied(points, r)
    act = np.zeros_like(occ)
    for z, y, x in zip(*np.nonzero(occ)):
        act[max(z - halo, 0):z + halo + 1, max(y - halo, 0):y + halo + 1,
            max(x - halo, 0):x + halo + 1] = True
    return act


def stack_masks(points: np.ndarray, res, halo: int = HALO, span: int = 2) -> list:
    """Masks of every stack b = 0 .. F - span: stack b is pruned by frames
    b .. b + span - 1 of points (F, 3, N).  Returns [stack][level] of [r, r, r]."""
    f = np.asarray(points).shape[0]
    return [[active_mask([points[b + k] for k in range(span)], r, halo) for r in res]
            for b in range(f - span + 1)]


def induced_laplacian(r: int, mask: np.ndarray) -> sp.csr_matrix:
    """L_S of the cells where mask ([r, r, r], flat index (z r + y) r + x) is
    true, in the order of their flat indices."""
    keep = np.flatnonzero(np.asarray(mask, dtype=bool).reshape(-1))
    box = _pc.laplacian(r)
    adj = (sp.diags(box.diagonal()) - box).tocsr()[keep][:, keep]
    deg = np.asarray(adj.sum(axis=1)).reshape(-1)
    return (sp.diags(deg) - adj).tocsr()


def apply_masked(g: np.ndarray, r: int, lam: float, mask: np.ndarray) -> np.ndarray:
    """(I + lam L_S)^{-2} on the kept cells of every row of g (..., r^3), zero
    on the pruned ones (float64)."""
    g = np.asarray(g, dtype=np.float64)
    keep = np.flatnonzero(np.asarray(mask, dtype=bool).reshape(-1))
    flat = g.reshape(-1, r ** 3)
    out = np.zeros_like(flat)
    if keep.size:
        lu = spla.splu((sp.identity(keep.size) + lam * induced_laplacian(r, mask)).tocsc())
        for b in range(flat.shape[0]):
            out[b, keep] = lu.solve(lu.solve(flat[b, keep]))
    return out.reshape(g.shape)


def apply_levels_masked(flat: np.ndarray, res, lams, masks, channels: int = 3) -> np.ndarray:
    """Precondition one transition's packed gradient level by level on its
    pruned grids (masks: one [r, r, r] per level); every channel of a level
    (three, or the six of the cells [z; t] of Eq. 4-7) on the same kept cells."""
    out, off = [], 0
    flat = np.asarray(flat, dtype=np.float64)
    for r, lam, mk in zip(res, lams, masks):
        n = channels * r ** 3
        out.append(apply_masked(flat[off:off + n].reshape(channels, r ** 3), r, lam, mk).reshape(-1))
        off += n
    return np.concatenate(out)


def packed_mask(masks, res, channels: int = 3) -> np.ndarray:
    """Boolean over one transition's packed values (``channels`` per level)."""
    return np.concatenate([np.tile(np.asarray(mk, bool).reshape(-1), channels)
                           for mk, _ in zip(masks, res)])
