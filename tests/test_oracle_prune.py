"""Pins for the oracle's pruned grids (Sec. 3.6).

* cells of points: cell centres, the cube's faces and points outside it;
* the active set against scipy's binary dilation with a 3x3x3 structuring
  element repeated halo times (the Chebyshev ball), and hand counts (a cube of
  7^3 cells in the middle, 4^3 in a corner);
* the preconditioner on the induced graph: the full mask gives the box's DCT
  closed form; a cube-shaped mask gives the DCT closed form of the smaller
  cube (the induced graph of a sub-box is a box); two cubes with a gap are
  solved independently; pruned cells come out zero; constants on a connected
  kept set pass unchanged; the operator is symmetric;
* six-channel cells (Eq. 4-7) on pruned grids: every one of the six channels
  of a level is preconditioned on the same kept cells -- full masks give the
  box's DCT closed form of all six channels, cube masks the DCT of the
  sub-cubes, pruned values come out zero, and a full step with full masks
  equals the unpruned six-channel step.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import precond as PC
from oracle import prune as PR


def test_cell_index():
    r = 8
    centres = -1.0 + (np.arange(r) + 0.5) * 2.0 / r
    x = np.stack([centres, centres[::-1], np.full(r, 0.1)])
    i = PR.cell_index(x, r)
    assert i[0].tolist() == list(range(r))
    assert i[1].tolist() == list(range(r))[::-1]
    assert set(i[2].tolist()) == {4}
    # faces and outside points clamp to the border cells
    e = PR.cell_index(np.array([[-1.0, 1.0, -3.0, 2.0]] * 3), r)
    assert e[0].tolist() == [0, r - 1, 0, r - 1]


def test_active_mask_counts():
    r = 16
    mid = np.full((3, 1), 0.01)
    assert PR.active_mask([mid], r).sum() == 7 ** 3
    assert PR.active_mask([mid], r, halo=0).sum() == 1
    assert PR.active_mask([mid], r, halo=1).sum() == 27
    corner = np.full((3, 1), -0.999)
    assert PR.active_mask([corner], r).sum() == 4 ** 3
    far = np.array([[-0.6, 0.6], [-0.6, 0.6], [-0.6, 0.6]])
    assert PR.active_mask([far], r).sum() == 2 * 7 ** 3


@pytest.mark.parametrize("r,halo", [(8, 3), (16, 3), (12, 2), (5, 1)])
def test_active_mask_is_binary_dilation(r, halo):
    rng = np.random.default_rng(r + halo)
    pts = [rng.uniform(-1.1, 1.1, (3, 40)).astype(np.float32),
           rng.normal(0, 0.3, (3, 30)).astype(np.float32)]
    occ = PR.occupied(pts, r)
    ref = ndimage.binary_dilation(occ, structure=np.ones((3, 3, 3), bool), iterations=halo)
    np.testing.assert_array_equal(PR.active_mask(pts, r, halo), ref)


def test_full_mask_is_dct():
    r, lam = 6, 0.4
    g = np.random.default_rng(1).normal(size=(3, r ** 3))
    full = np.ones((r, r, r), bool)
    np.testing.assert_allclose(PR.apply_masked(g, r, lam, full), PC.apply_dct(g, r, lam),
                               atol=1e-12)


def _embed(r, boxes, g_sub):
    out = np.zeros((g_sub[0].shape[0], r, r, r))
    for (z, y, x, s), gs in zip(boxes, g_sub):
        out[:, z:z + s, y:y + s, x:x + s] = gs.reshape(-1, s, s, s)
    return out.reshape(-1, r ** 3)


def test_cube_masks_reduce_to_dct_of_the_cube():
    r, lam = 10, 0.7
    rng = np.random.default_rng(2)
    boxes = [(1, 2, 0, 4), (5, 5, 6, 3)]          # (z0, y0, x0, side); gap between them
    mask = np.zeros((r, r, r), bool)
    for z, y, x, s in boxes:
        mask[z:z + s, y:y + s, x:x + s] = True
    g = rng.normal(size=(2, r ** 3))
    got = PR.apply_masked(g, r, lam, mask)
    subs = []
    for z, y, x, s in boxes:
        gs = g.reshape(2, r, r, r)[:, z:z + s, y:y + s, x:x + s].reshape(2, -1)
        subs.append(PC.apply_dct(gs, s, lam))
    np.testing.assert_allclose(got, _embed(r, boxes, subs), atol=1e-12)


def test_zero_outside_constants_symmetry():
    r, lam = 8, 1.3
    rng = np.random.default_rng(3)
    mask = PR.active_mask([rng.normal(0, 0.2, (3, 5)).astype(np.float32)], r, halo=1)
    lab, ncomp = ndimage.label(mask)
    g = rng.normal(size=(1, r ** 3))
    out = PR.apply_masked(g, r, lam, mask)
    assert np.all(out[0, ~mask.reshape(-1)] == 0.0)
    for c in range(1, ncomp + 1):
        ones = (lab == c).reshape(1, -1).astype(np.float64)
        comp_only = PR.apply_masked(ones, r, lam, mask)
        np.testing.assert_allclose(comp_only, ones, atol=1e-12)
    a, b = rng.normal(size=(1, r ** 3)), rng.normal(size=(1, r ** 3))
    pa, pb = PR.apply_masked(a, r, lam, mask), PR.apply_masked(b, r, lam, mask)
    assert abs(np.sum(pa * b) - np.sum(a * pb)) <= 1e-12 * np.sum(np.abs(a * b))


def test_stack_masks_use_both_frames():
    rng = np.random.default_rng(4)
    pts = rng.uniform(-1, 1, (3, 3, 20)).astype(np.float32)
    ms = PR.stack_masks(pts, [8], halo=0, span=2)
    assert len(ms) == 2
    for b in range(2):
        np.testing.assert_array_equal(ms[b][0], PR.occupied([pts[b], pts[b + 1]], 8))


PAPER_RES = (1, 3, 5, 7)               # R = 2l - 1, the first levels of the paper's grid


def _lams(res):
    return [0.25 * 1.5 ** l for l in range(len(res))]


def test_six_channel_full_masks_are_dct():
    res = PAPER_RES
    g = np.random.default_rng(21).normal(size=6 * sum(r ** 3 for r in res))
    full = [np.ones((r, r, r), bool) for r in res]
    got = PR.apply_levels_masked(g, res, _lams(res), full, channels=6)
    ref = PC.apply_levels(g, res, _lams(res), "dct", channels=6)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_six_channel_cube_masks_and_zeros():
    res = (4, 9)
    rng = np.random.default_rng(22)
    boxes = {4: [(0, 1, 1, 3)], 9: [(1, 2, 0, 4), (5, 5, 5, 3)]}
    masks = []
    for r in res:
        m = np.zeros((r, r, r), bool)
        for z, y, x, sd in boxes[r]:
            m[z:z + sd, y:y + sd, x:x + sd] = True
        masks.append(m)
    lams = _lams(res)
    g = rng.normal(size=6 * sum(r ** 3 for r in res))
    got = PR.apply_levels_masked(g, res, lams, masks, channels=6)
    keep = PR.packed_mask(masks, res, channels=6)
    assert keep.size == got.size and np.all(got[~keep] == 0.0)
    off = 0
    for r, lam in zip(res, lams):
        gl = g[off:off + 6 * r ** 3].reshape(6, r, r, r)
        subs = [PC.apply_dct(gl[:, z:z + sd, y:y + sd, x:x + sd].reshape(6, -1), sd, lam)
                for z, y, x, sd in boxes[r]]
        np.testing.assert_allclose(got[off:off + 6 * r ** 3],
                                   _embed(r, boxes[r], subs).reshape(-1), atol=1e-12)
        off += 6 * r ** 3


def test_six_channel_step_full_masks_equal_unpruned():
    import synth
    from oracle import sequence as S
    res = (1, 3)
    seq = synth.deforming_sequence(seed=23, frames=3, n=60, subdiv=0)
    P6 = 6 * sum(r ** 3 for r in res)
    theta = np.random.default_rng(24).normal(0, 0.05, (2, P6))
    z = np.zeros_like(theta)
    full = [[np.ones((r, r, r), bool) for r in res] for _ in range(2)]
    hp = S.Hyper(e_max=10)
    a = S.step(seq.points, seq.template, seq.edges, res, theta, z, z, 1, hp, channels=6)
    b = S.step(seq.points, seq.template, seq.edges, res, theta, z, z, 1, hp, channels=6,
               masks=full)
    np.testing.assert_allclose(b.pgrad, a.pgrad, atol=1e-12 * np.abs(a.pgrad).max())
    np.testing.assert_allclose(b.theta, a.theta, atol=1e-12)
