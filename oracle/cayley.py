"""Six-channel cells with the Cayley rotation (paper Sec. 3.3, Eq. 4-7) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each cell stores T = [z; t] (Eq. 4): z parameterises a rotation through the
Cayley map R(z) = (I + Z)(I - Z)^{-1} (Eq. 5) of the skew-symmetric matrix Z
built from z (Eq. 6), and t is a translation.  The transformation at a point
is the level average of the trilinearly interpolated cell vectors (Eq. 1), and
the point moves by the homogeneous transform of Eq. 7:

    x' = R(z^(x)) x + t^(x),   [z^; t^](x) = level_scale * sum_l trilerp(G_l, x).

With z = 0 everywhere R = I and this is the translation warp of ``warp``.

Readings (the paper does not state them):
* Channel order inside a level: z_0, z_1, z_2, t_x, t_y, t_z (the order of
  Eq. 4); a level is a float array (6, R, R, R) indexed [c, z, y, x], levels
  packed one after the other.
* R acts on the point's coordinates in the normalised cube, i.e. about the
  origin (Eq. 7 applies M to the point itself).
* Cell centres, border clamp, R = 1 levels and level_scale as in ``warp``.

Everything here is float64 and follows the definitions literally: R by a
3 x 3 inverse per point, its derivative by differentiating Eq. 5 as a matrix
product (dR = (I + R) dZ (I - Z)^{-1}).
"""
from __future__ import annotations

import numpy as np

from . import warp as W

CH = 6


def skew(z: np.ndarray) -> np.ndarray:
    """Z of Eq. 6 for every column of z (3, n): array (n, 3, 3)."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[1]
    m = np.zeros((n, 3, 3))
    m[:, 0, 1], m[:, 0, 2] = -z[2], z[1]
    m[:, 1, 0], m[:, 1, 2] = z[2], -z[0]
    m[:, 2, 0], m[:, 2, 1] = -z[1], z[0]
    return m


def cayley(z: np.ndarray) -> np.ndarray:
    """R(z) = (I + Z)(I - Z)^{-1} (Eq. 5) for every column of z: (n, 3, 3)."""
    zm = skew(z)
    eye = np.eye(3)[None]
    return (eye + zm) @ np.linalg.inv(eye - zm)


def dcayley(z: np.ndarray) -> np.ndarray:
    """dR/dz_k for every column of z: array (n, 3, 3, 3) indexed [i, k].

    Differentiating Eq. 5 with d(I - Z)^{-1} = (I - Z)^{-1} dZ (I - Z)^{-1}
    gives dR = dZ (I - Z)^{-1} + (I + Z)(I - Z)^{-1} dZ (I - Z)^{-1}
             = (I + R) dZ (I - Z)^{-1}, with dZ = skew(e_k) for z_k."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[1]
    eye = np.eye(3)[None]
    inv = np.linalg.inv(eye - skew(z))
    r = cayley(z)
    out = np.empty((n, 3, 3, 3))
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = 1.0
        ek = skew(e)                       # (1, 3, 3)
        out[:, k] = (eye + r) @ ek @ inv
    return out


def unpack(flat: np.ndarray, res) -> list:
    """Split a packed six-channel stack into per-level (6, R, R, R) views."""
    out, off = [], 0
    for r in res:
        n = CH * r ** 3
        out.append(np.asarray(flat[off:off + n]).reshape(CH, r, r, r))
        off += n
    if off != np.asarray(flat).shape[0]:
        raise ValueError("packed grid size does not match resolutions")
    return out


def grid_size(res) -> int:
    return CH * sum(int(r) ** 3 for r in res)


def transform(flat: np.ndarray, res, x: np.ndarray, level_scale: float) -> np.ndarray:
    """[z^; t^](x) = level_scale * sum_l trilerp(G_l, x) (Eq. 1): (6, n)."""
    x = np.asarray(x, dtype=np.float64)
    t = np.zeros((CH, x.shape[1]))
    for g, r in zip(unpack(np.asarray(flat, np.float64), res), res):
        a = W.interp_matrix(r, x)
        gl = g.reshape(CH, -1)
        for c in range(CH):
            t[c] += a @ gl[c]
    return level_scale * t


def warp6(flat: np.ndarray, res, x: np.ndarray, level_scale: float) -> np.ndarray:
    """x' = R(z^(x)) x + t^(x) (Eq. 1, 5-7): float64 (3, n)."""
    x = np.asarray(x, dtype=np.float64)
    t = transform(flat, res, x, level_scale)
    r = cayley(t[:3])
    return np.einsum("nij,jn->in", r, x) + t[3:]


def lam6(flat: np.ndarray, res, x: np.ndarray, gout: np.ndarray,
         level_scale: float) -> np.ndarray:
    """Adjoint of the interpolated cell vector for an upstream gradient gout of
    x': d<gout, x'>/dz^_k = gout . (dR/dz_k x), d<gout, x'>/dt^ = gout. (6, n)."""
    x = np.asarray(x, dtype=np.float64)
    gout = np.asarray(gout, dtype=np.float64)
    t = transform(flat, res, x, level_scale)
    dr = dcayley(t[:3])                       # (n, k, i, j)
    u = np.einsum("in,nkij,jn->kn", gout, dr, x)
    return np.concatenate([u, gout])


def grid_adjoint6(flat: np.ndarray, res, x: np.ndarray, gout: np.ndarray,
                  level_scale: float) -> np.ndarray:
    """Gradient of <gout, warp6(G, x)> with respect to the packed values:
    level_scale * A_l^T lam_c per level and channel (transpose of Eq. 1)."""
    lam = lam6(flat, res, x, gout, level_scale)
    parts = []
    for r in res:
        a = W.interp_matrix(r, x)
        parts.append(np.stack([level_scale * (a.T @ lam[c]) for c in range(CH)]).reshape(-1))
    return np.concatenate(parts)


def interp_gradient(g: np.ndarray, r: int, x: np.ndarray) -> np.ndarray:
    """d/dx of trilerp(g_c, x) for a level g (C, r, r, r): array (C, 3, n).

    Along axis a the derivative is (r/2) times the difference of the two faces
    of the stencil, weighted by the other two axes; it is zero along an axis
    whose coordinate was clamped (as in ``warp.position_adjoint``)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[1]
    c = g.shape[0]
    out = np.zeros((c, 3, n))
    if r == 1:
        return out
    idx, w, f, inside, _ = W.corner_weights(r, x)
    gl = np.asarray(g, np.float64).reshape(c, -1)
    for a in range(3):
        dw = np.empty_like(w)
        for k in range(8):
            d = (k & 1, (k >> 1) & 1, (k >> 2) & 1)
            t = np.ones(n)
            for b in range(3):
                if b == a:
                    t = t * (1.0 if d[b] else -1.0)
                else:
                    t = t * (f[b] if d[b] else 1.0 - f[b])
            dw[:, k] = t
        for ch in range(c):
            out[ch, a] = (r / 2.0) * inside[a] * np.sum(dw * gl[ch][idx], axis=1)
    return out


def position_adjoint6(flat: np.ndarray, res, x: np.ndarray, gout: np.ndarray,
                      level_scale: float) -> np.ndarray:
    """Gradient of <gout, warp6(G, x)> with respect to x: R^T gout plus the
    chain through the interpolated cell vector, sum_c lam_c grad T^_c. (3, n)."""
    x = np.asarray(x, dtype=np.float64)
    gout = np.asarray(gout, dtype=np.float64)
    t = transform(flat, res, x, level_scale)
    r = cayley(t[:3])
    gx = np.einsum("nij,in->jn", r, gout)
    lam = lam6(flat, res, x, gout, level_scale)
    for g, rr in zip(unpack(np.asarray(flat, np.float64), res), res):
        grad = interp_gradient(g, rr, x)           # (6, 3, n)
        gx += level_scale * np.einsum("cn,can->an", lam, grad)
    return gx
