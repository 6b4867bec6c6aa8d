"""Multi-resolution trilinear deformation (paper Sec. 3.1, Eq. 1) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 1 gives the transformation at a point as the average over the L levels
of the trilinearly interpolated cell values.  The hot path stores a
3-channel translation per cell (the Cayley rotation of Eq. 4-7 with z = 0,
where R(0) = I and the homogeneous transform of Eq. 7 reduces to x + t), so

    warp(x) = x + level_scale * sum_l trilerp(G_l, x),   level_scale = 1/L.

Readings (the paper does not state them):
* Cell-centred values on the domain [-1, 1]^3 (Sec. 3.6 normalises the
  points to this cube): the centre of cell i of a level with R cells per axis
  is -1 + (2 i + 1) / R.
* Points outside the hull of the centres are clamped to it per axis (border
  clamp), so the weights always sum to one.
* A level with R = 1 is a single constant transform.

Layout of a grid level: float array (3, R, R, R) indexed [c, z, y, x]; a
transition packs its levels one after the other (``pack`` / ``unpack``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def unpack(flat: np.ndarray, res) -> list:
    """Split one transition's packed values into per-level (3, R, R, R) views."""
    out, off = [], 0
    for r in res:
        n = 3 * r ** 3
        out.append(np.asarray(flat[off:off + n]).reshape(3, r, r, r))
        off += n
    if off != flat.shape[0]:
        raise ValueError("packed grid size does not match resolutions")
    return out


def pack(levels) -> np.ndarray:
    return np.concatenate([np.asarray(g).reshape(-1) for g in levels])


def corner_weights(r: int, x: np.ndarray):
    """Trilinear stencil of samples x (3, n) in a level with r cells per axis.

    Returns (idx (n, 8) flat node index into r^3 with x fastest,
             w (n, 8) float64 weights,
             f (3, n) fractional coordinates,
             inside (3, n) bool: the axis coordinate was not clamped,
             i0 (3, n) base cell).
    Corner k has offsets (dx, dy, dz) = (k & 1, (k >> 1) & 1, (k >> 2) & 1).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    if r == 1:
        return (np.zeros((n, 8), np.int64), np.tile([1.0] + [0.0] * 7, (n, 1)),
                np.zeros((3, n)), np.zeros((3, n), bool), np.zeros((3, n), np.int64))
    u = (x + 1.0) * (r / 2.0) - 0.5
    inside = (u >= 0.0) & (u <= r - 1.0)
    uc = np.clip(u, 0.0, r - 1.0)
    i0 = np.minimum(np.floor(uc), r - 2).astype(np.int64)
    f = uc - i0
    idx = np.empty((n, 8), np.int64)
    w = np.empty((n, 8), np.float64)
    for k in range(8):
        d = (k & 1, (k >> 1) & 1, (k >> 2) & 1)
        wk = np.ones(n)
        for a in range(3):
            wk = wk * (f[a] if d[a] else 1.0 - f[a])
        w[:, k] = wk
        idx[:, k] = ((i0[2] + d[2]) * r + (i0[1] + d[1])) * r + (i0[0] + d[0])
    return idx, w, f, inside, i0


def interp_matrix(r: int, x: np.ndarray) -> sp.csr_matrix:
    """Sparse (n, r^3) matrix A with (A g)[i] = trilerp(g, x_i) (Eq. 1, one level)."""
    idx, w, *_ = corner_weights(r, x)
    n = idx.shape[0]
    rows = np.repeat(np.arange(n), 8)
    return sp.csr_matrix((w.reshape(-1), (rows, idx.reshape(-1))), shape=(n, r ** 3))


def displacement(levels, res, x: np.ndarray, level_scale: float) -> np.ndarray:
    """D(x) = level_scale * sum_l trilerp(G_l, x), float64 (3, n)."""
    x = np.asarray(x, dtype=np.float64)
    d = np.zeros_like(x)
    for g, r in zip(levels, res):
        a = interp_matrix(r, x)
        gl = np.asarray(g, dtype=np.float64).reshape(3, -1)
        for c in range(3):
            d[c] += a @ gl[c]
    return level_scale * d


def warp(flat: np.ndarray, res, x: np.ndarray, level_scale: float) -> np.ndarray:
    """Deformed positions x + D(x) (Eq. 1 with the translation form of Eq. 7)."""
    x = np.asarray(x, dtype=np.float64)
    return x + displacement(unpack(np.asarray(flat, np.float64), res), res, x, level_scale)


def grid_adjoint(res, x: np.ndarray, gout: np.ndarray, level_scale: float) -> np.ndarray:
    """Gradient of <gout, warp(G, x)> with respect to the packed grid values:
    level_scale * A_l^T gout_c per level and channel (transpose of Eq. 1)."""
    gout = np.asarray(gout, dtype=np.float64)
    parts = []
    for r in res:
        a = interp_matrix(r, x)
        parts.append(np.stack([level_scale * (a.T @ gout[c]) for c in range(3)]).reshape(-1))
    return np.concatenate(parts)


def position_adjoint(flat: np.ndarray, res, x: np.ndarray, gout: np.ndarray,
                     level_scale: float) -> np.ndarray:
    """J^T gout for out = x + D(x): gout + (dD/dx)^T gout, float64 (3, n).

    The derivative of a trilinear interpolant along axis a is (R/2) times the
    difference of the two faces, weighted by the other two axes; it is zero
    along an axis whose coordinate was clamped, and the base-cell convention
    makes it one-sided exactly on interior cell-centre planes.
    """
    x = np.asarray(x, dtype=np.float64)
    gout = np.asarray(gout, dtype=np.float64)
    gx = gout.copy()
    for g, r in zip(unpack(np.asarray(flat, np.float64), res), res):
        if r == 1:
            continue
        idx, w, f, inside, _ = corner_weights(r, x)
        gl = g.reshape(3, -1)
        # s_k = sum_c gout_c * G_c[corner k]
        s = np.zeros_like(w)
        for c in range(3):
            s += gout[c][:, None] * gl[c][idx]
        for a in range(3):
            dw = np.empty_like(w)
            for k in range(8):
                d = (k & 1, (k >> 1) & 1, (k >> 2) & 1)
                t = np.ones(x.shape[1])
                for b in range(3):
                    if b == a:
                        t = t * (1.0 if d[b] else -1.0)
                    else:
                        t = t * (f[b] if d[b] else 1.0 - f[b])
                dw[:, k] = t
            gx[a] += level_scale * (r / 2.0) * inside[a] * np.sum(dw * s, axis=1)
    return gx
