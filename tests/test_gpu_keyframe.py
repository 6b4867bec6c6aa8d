"""GPU parity of keyframe selection (Sec. 3.5, Eq. 19-20) against the oracle:
occupied-voxel counts and the selected frame are integers, compared exactly."""
import numpy as np
import pytest
import torch

import synth
from oracle import keyframe as K
from paper_2509_18097_amd import _lib as L
from _gpu import dev, host, require_gpu

pytestmark = pytest.mark.gpu


def _check(points, gamma=0.001):
    key, counts = L.keyframe(dev(points), gamma)
    rk, rc = K.keyframe(points, gamma)
    assert np.array_equal(host(counts), rc)
    assert int(host(key)[0]) == rk
    return rk


def test_sequence_32_frames_50k_points():
    """The headline sequence's frames (32 x 50,000 points on a deforming ellipsoid)."""
    require_gpu()
    seq = synth.deforming_sequence(seed=0, frames=32, n=50_000, subdiv=2)
    _check(seq.points)


def test_boundaries_clamps_and_duplicates():
    require_gpu()
    rng = np.random.default_rng(1)
    f, n = 7, 3001
    pts = rng.uniform(-1.2, 1.2, (f, 3, n)).astype(np.float32)
    # exact voxel faces, the cube's faces and beyond, repeated points
    faces = (np.arange(-64, 65) / 64.0).astype(np.float32)
    pts[:, :, :faces.size] = faces[None, None, :]
    pts[2, :, :1500] = pts[2, :, :1]
    pts[3] = np.float32(0.5)                         # one voxel
    _check(pts)


def test_weighting_and_ties_and_empty():
    require_gpu()
    n = 1000
    rng = np.random.default_rng(2)
    cells = rng.choice(128 ** 3, size=n, replace=False)
    centres = lambda ids: np.stack([((ids // 128 ** e) % 128 + 0.5) / 64.0 - 1.0
                                    for e in range(3)]).astype(np.float32)
    frames = np.zeros((101, 3, n), np.float32)
    frames[:] = centres(np.repeat(cells[:1], n))
    frames[0] = centres(cells)
    frames[50] = centres(np.concatenate([cells[:990], np.repeat(cells[:1], 10)]))
    assert _check(frames) == 50
    assert _check(frames, gamma=0.0) == 0
    assert _check(np.zeros((4, 3, 8), np.float32)) == 1          # ties: the earliest frame
    key, counts = L.keyframe(torch.zeros((5, 3, 0), dtype=torch.float32, device="cuda"))
    assert host(counts).tolist() == [0] * 5 and int(host(key)[0]) == 0
