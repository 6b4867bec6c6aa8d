"""Robust Chamfer distance (paper Sec. 3.4, Eq. 11-13) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

CD_R(P, Q) = 1/|P| sum_p w(p, q_p) |p - q_p|^2 + 1/|Q| sum_q w(p_q, q) |p_q - q|^2,
with q_p, p_q the nearest neighbours in the other set (Eq. 12) and the
Gaussian weight w(p, q) = exp(-alpha |p - q|^2), alpha = 5.56 (Eq. 13).

Readings:
* Nearest neighbours are found by brute force over all pairs.  Ties go to the
  lowest index.  The index contract for float32 inputs is the squared
  distance evaluated in float32 in difference form with no fused multiply-add:
      dx = fl(a_x - b_x), ... ;  d2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)).
  (``nn_fp32``).  The float64 argmin (``nn_fp64``) is available for reporting
  how often rounding changes the neighbour.
* The loss is accumulated in float64 from float64 distances of the float32
  coordinates.
* The weight w_R is differentiated (the paper marks stop-gradients explicitly
  elsewhere, Eq. 17, and not here), so d/ds [exp(-alpha s) s] =
  exp(-alpha s) (1 - alpha s).  The second set (the observed points) is data
  and receives no gradient.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

ALPHA = 5.56          # Eq. 13


def _nn_chunk(a, b, lo, hi, dtype):
    ax = a[0, lo:hi, None].astype(dtype)
    ay = a[1, lo:hi, None].astype(dtype)
    az = a[2, lo:hi, None].astype(dtype)
    dx = ax - b[0][None, :].astype(dtype)
    dy = ay - b[1][None, :].astype(dtype)
    dz = az - b[2][None, :].astype(dtype)
    d2 = (dx * dx + dy * dy) + dz * dz
    return np.argmin(d2, axis=1)           # first occurrence = lowest index


def _nn(a, b, dtype, chunk, workers):
    a = np.asarray(a)
    b = np.asarray(b)
    n = a.shape[1]
    if n == 0 or b.shape[1] == 0:
        raise ValueError("Chamfer needs two non-empty point sets (Eq. 11 divides by |P|, |Q|)")
    starts = list(range(0, n, chunk))
    if workers <= 1 or len(starts) == 1:
        parts = [_nn_chunk(a, b, s, min(n, s + chunk), dtype) for s in starts]
    else:
        with ThreadPoolExecutor(workers) as ex:
            parts = list(ex.map(lambda s: _nn_chunk(a, b, s, min(n, s + chunk), dtype), starts))
    return np.concatenate(parts).astype(np.int64)


def nn_fp32(a, b, chunk: int = 256, workers: int = 1) -> np.ndarray:
    """Index of the nearest point of b for every point of a (Eq. 12), float32
    difference-form contract, lowest index on ties.  a (3, n), b (3, m) float32."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    return _nn(a, b, np.float32, chunk, workers)


def nn_fp64(a, b, chunk: int = 256, workers: int = 1) -> np.ndarray:
    """As ``nn_fp32`` but with the distances in float64."""
    return _nn(np.asarray(a, np.float64), np.asarray(b, np.float64), np.float64, chunk, workers)


def sqdist(a, b, nn) -> np.ndarray:
    """|a_i - b_nn[i]|^2 in float64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = a - b[:, nn]
    return np.sum(d * d, axis=0)


def direction_loss(a, b, nn_a, alpha: float = ALPHA) -> float:
    """1/|A| sum_i exp(-alpha s_i) s_i with s_i = |a_i - b_nn_a[i]|^2 (one term of Eq. 11)."""
    s = sqdist(a, b, nn_a)
    return float(np.mean(np.exp(-alpha * s) * s))


def chamfer(a, b, alpha: float = ALPHA, workers: int = 1):
    """Both directions of CD_R(A, B).  Returns (loss_ab, loss_ba, nn_a, nn_b)
    with nn_a[i] in B for each a_i and nn_b[j] in A for each b_j."""
    nn_a = nn_fp32(a, b, workers=workers)
    nn_b = nn_fp32(b, a, workers=workers)
    return direction_loss(a, b, nn_a, alpha), direction_loss(b, a, nn_b, alpha), nn_a, nn_b


def gradient(a, b, nn_a, nn_b, alpha: float = ALPHA, w_ab: float = 1.0,
             w_ba: float = 1.0) -> np.ndarray:
    """d/da of w_ab * loss_ab + w_ba * loss_ba with the assignment frozen.

    Forward term:  w_ab/|A| * e^{-alpha s}(1 - alpha s) * 2 (a_i - b_nn_a[i]).
    Reverse term:  for every b_j, w_ba/|B| * e^{-alpha s_j}(1 - alpha s_j)
                   * 2 (a_nn_b[j] - b_j) added to a_nn_b[j].
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n, m = a.shape[1], b.shape[1]
    g = np.zeros_like(a)
    d = a - b[:, nn_a]
    s = np.sum(d * d, axis=0)
    g += (w_ab / n) * (np.exp(-alpha * s) * (1.0 - alpha * s))[None, :] * 2.0 * d
    d2 = a[:, nn_b] - b
    s2 = np.sum(d2 * d2, axis=0)
    contrib = (w_ba / m) * (np.exp(-alpha * s2) * (1.0 - alpha * s2))[None, :] * 2.0 * d2
    for c in range(3):
        np.add.at(g[c], nn_b, contrib[c])
    return g
