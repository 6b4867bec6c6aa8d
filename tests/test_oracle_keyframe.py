"""Pins for the oracle's keyframe selection (Sec. 3.5, Eq. 19-20): voxel
boundaries placed by hand, occupancy counted by hand, the Gaussian weight's
closed form, and winners decided by the weighting."""
import numpy as np

from oracle import keyframe as K


def test_voxel_boundaries():
    # voxel i covers [-1 + i/64, -1 + (i+1)/64); the cube's faces clamp
    x = np.array([[-1.0, -1.0 + 1.0 / 64, -1.0 + 1.0 / 64 - 2.0 ** -20, 0.0, -2.0 ** -20,
                   1.0 - 2.0 ** -20, 1.0, 3.0, -5.0]], np.float32)
    pts = np.concatenate([x, np.full_like(x, -1.0), np.full_like(x, -1.0)])
    assert K.voxel_ids(pts).tolist() == [0, 1, 0, 64, 63, 127, 127, 127, 0]
    # y and z strides
    p = np.array([[-1.0], [-1.0 + 3.0 / 64], [-1.0 + 5.0 / 64]], np.float32)
    assert K.voxel_ids(p).tolist() == [(5 * 128 + 3) * 128 + 0]


def test_occupancy_counts_distinct_voxels():
    a = np.tile(np.array([[0.1], [0.2], [0.3]], np.float32), (1, 10))   # one voxel, 10 points
    b = np.array([[-0.9 + 0.1 * k for k in range(5)], [0.0] * 5, [0.0] * 5], np.float32)
    c = np.concatenate([b[:, :3], b[:, :3]], axis=1)                     # 3 voxels, twice each
    frames = np.stack([np.pad(m, ((0, 0), (0, 10 - m.shape[1])), mode="edge") for m in (a, b, c)])
    assert K.occupancy(frames).tolist() == [1, 5, 3]


def test_weights_closed_form():
    w = K.weights(5, 0.001)
    # T = 4, centre 2: exp(-0.001 * {4, 1, 0, 1, 4})
    np.testing.assert_allclose(w, np.exp(-0.001 * np.array([4.0, 1.0, 0.0, 1.0, 4.0])), rtol=0,
                               atol=0)


def test_weighting_decides_the_winner():
    # 101 frames: frame 0 covers 1000 voxels, the centre frame 990: the weight
    # exp(-0.001 * 50^2) = 0.082 makes the centre win; with gamma = 0 frame 0 wins
    rng = np.random.default_rng(0)
    n = 1000
    frames = np.zeros((101, 3, n), np.float32)
    cells = rng.choice(128 ** 3, size=n, replace=False)
    centres = lambda ids: np.stack([((ids // 128 ** e) % 128 + 0.5) / 64.0 - 1.0 for e in range(3)])
    frames[0] = centres(cells)
    frames[50] = centres(np.concatenate([cells[:990], np.repeat(cells[:1], 10)]))
    for t in range(101):
        if t not in (0, 50):
            frames[t] = centres(np.repeat(cells[:1], n))
    key, counts = K.keyframe(frames)
    assert counts[0] == 1000 and counts[50] == 990 and counts[1] == 1
    assert key == 50
    assert K.keyframe(frames, gamma=0.0)[0] == 0


def test_ties_go_to_the_earliest_frame():
    f = np.zeros((4, 3, 8), np.float32)            # every frame: one voxel
    assert K.keyframe(f)[0] == 1                    # T = 3: frames 1 and 2 tie, 1 wins
