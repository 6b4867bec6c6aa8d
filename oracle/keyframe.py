"""Keyframe selection (paper Sec. 3.5, Eq. 19-20) -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The keyframe is the frame with the largest number of occupied voxels of a
fixed 128^3 grid, weighted by a Gaussian in the distance of its index from
the temporal midpoint:

    t_key = argmax_t  exp(-gamma (t - T/2)^2) * |G(P_t)|,   gamma = 0.001,

over the frames t = 0..T (T = F - 1 for F frames).

Readings (the paper does not state them):
* The 128^3 grid covers the normalised cube [-1, 1]^3 (Sec. 3.6 normalises the
  points to it): voxel i along an axis holds -1 + i/64 <= x < -1 + (i+1)/64;
  coordinates outside the cube, and x = 1 itself, are clamped to the border
  voxels 0 and 127.
* Ties of the weighted score go to the earliest frame.
* The voxel of a coordinate is decided in float32, (x + 1) * 64 rounded to
  nearest then floored (the multiplication by 64 is exact), as the GPU
  decides it; the score is evaluated in float64.
"""
from __future__ import annotations

import numpy as np

GRID = 128
GAMMA = 0.001


def voxel_ids(x: np.ndarray) -> np.ndarray:
    """Flat voxel index (x fastest) of every column of x (3, n)."""
    x = np.asarray(x, dtype=np.float32)
    u = (x + np.float32(1.0)) * np.float32(GRID / 2)          # float32, as decided on the GPU
    i = np.clip(np.floor(u.astype(np.float64)), 0, GRID - 1).astype(np.int64)
    return (i[2] * GRID + i[1]) * GRID + i[0]


def occupancy(points: np.ndarray) -> np.ndarray:
    """|G(P_t)| for every frame of points (F, 3, N): the number of distinct voxels."""
    return np.array([np.unique(voxel_ids(p)).size for p in points], dtype=np.int64)


def weights(frames: int, gamma: float = GAMMA) -> np.ndarray:
    """w_key(t - T/2) = exp(-gamma (t - T/2)^2) for t = 0..T, T = frames - 1 (Eq. 20)."""
    t = np.arange(frames, dtype=np.float64)
    return np.exp(-gamma * (t - (frames - 1) / 2.0) ** 2)


def keyframe(points: np.ndarray, gamma: float = GAMMA):
    """(t_key, counts) of Eq. 19 (first frame on ties)."""
    counts = occupancy(points)
    score = weights(points.shape[0], gamma) * counts.astype(np.float64)
    return int(np.argmax(score)), counts
