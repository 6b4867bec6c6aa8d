"""Pins for the oracle's Adam, isometry, confidence and full step."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import adam as A
from oracle import chamfer as C
from oracle import sequence as S
from oracle import warp as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_hyper_defaults_match_paper():
    h = S.Hyper()
    assert h.alpha == GOLD["alpha"]["value"] and h.w_iso == GOLD["w_iso"]["value"]
    assert (h.beta1, h.beta2, h.eps) == (GOLD["adam"]["beta1"], GOLD["adam"]["beta2"], GOLD["adam"]["eps"])
    etas, lams = h.schedule(5)
    assert etas[0] == GOLD["eta_level1"]["value"] and lams[0] == GOLD["lambda_level1"]["value"]
    np.testing.assert_allclose(etas[1] / etas[0], 1 + GOLD["eta_growth_per_level"]["value"])
    np.testing.assert_allclose(lams[1] / lams[0], 1 + GOLD["lambda_growth_per_level"]["value"])
    np.testing.assert_allclose(lams, [0.25, 0.375, 0.5625, 0.84375, 1.265625])


def test_adam_first_step_closed_form():
    # bias corrections cancel on the first step: update = -eta g / (|g| + eps)
    rng = np.random.default_rng(0)
    g = rng.normal(size=100) * 10.0 ** rng.uniform(-9, 1, 100)
    th, m, v = A.update(np.zeros(100), np.zeros(100), np.zeros(100), g, 0.01, 1)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_constant_gradient_and_zero_gradient():
    g = np.array([2.0, -3.0, 0.0])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for k in range(1, 6):
        prev = th.copy()
        th, m, v = A.update(th, m, v, g, 0.1, k)
        # with a constant gradient m^ = g and v^ = g^2 at every step
        np.testing.assert_allclose(th - prev, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert th[2] == 0.0


def test_isometry_rigid_motion_zero():
    v, f, e = synth.icosphere(2)
    x0 = v.T
    rng = np.random.default_rng(1)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    x1 = q @ x0 + np.array([[0.1], [0.2], [-0.3]])
    x2 = x1 + 0.5
    l_iso, g = S.isometry(np.stack([x0, x1, x2]), e)
    assert l_iso < 1e-14


def test_isometry_uniform_scale_closed_form():
    v, f, e = synth.icosphere(1)
    x0 = v.T
    s = 1.07
    l_iso, _ = S.isometry(np.stack([x0, s * x0]), e)
    ln = np.linalg.norm(x0[:, e[0]] - x0[:, e[1]], axis=0)
    assert abs(l_iso - abs(s - 1) * ln.mean()) < 1e-14


def test_isometry_gradient_finite_difference():
    v, f, e = synth.icosphere(1)
    rng = np.random.default_rng(2)
    x = np.stack([v.T + 0.05 * rng.normal(size=v.T.shape) for _ in range(4)])
    l0, g = S.isometry(x, e, 3.0)
    h = 1e-7
    for t in (1, 2, 3):
        for i in rng.choice(x.shape[2], 6, replace=False):
            for c in range(3):
                xp, xm = x.copy(), x.copy()
                xp[t, c, i] += h
                xm[t, c, i] -= h
                fd = (S.isometry(xp, e, 3.0)[0] - S.isometry(xm, e, 3.0)[0]) / (2 * h)
                assert abs(fd - g[t, c, i]) < 1e-6


def test_confidence_cases():
    # every template error below cd_max: all weights 1
    w, cdm, d = S.confidence([0.1, 0.2], [0.3, 0.25], epoch=3, e_max=50)
    assert cdm == 0.3 and np.all(w == 1.0)
    # at e = e_max the exponent is 0 and every weight is 1
    w, _, d = S.confidence([5.0, 7.0], [0.1, 0.1], epoch=50, e_max=50)
    assert d == 0.0 and np.all(w == 1.0)
    # hand-computed product at e = 0 (delta = 1): 1/(1+0.4) then 1/(1+0.4) * 1/(1+0.1)
    w, _, _ = S.confidence([0.5, 0.2], [0.1, 0.05], epoch=0, e_max=50)
    np.testing.assert_allclose(w, [1 / 1.4, 1 / 1.4 / 1.1], rtol=1e-15)


def _tiny_sequence(frames=4, n=60, subdiv=1, seed=0):
    return synth.deforming_sequence(seed=seed, frames=frames, n=n, subdiv=subdiv)


def test_step_fixed_point_exact():
    # zero grids, every frame identical and the template equal to the points:
    # every Chamfer term and the isometry term vanish, so the gradient is 0 and
    # Adam leaves the grids unchanged, exactly
    rng = np.random.default_rng(3)
    p = rng.uniform(-0.8, 0.8, (3, 50)).astype(np.float32)
    pts = np.stack([p] * 3)
    _, _, e = synth.icosphere(0)
    tmpl = p[:, :12].copy()
    res = (1, 2, 4)
    tot = 3 * sum(r ** 3 for r in res)
    z = np.zeros((2, tot))
    # tmpl points are a subset of p, so their NN distance is zero both ways
    # only when the template equals the cloud; use the cloud as template
    r = S.step(pts, p, np.array([[0], [1]], np.int32), res, z, z, z, epoch=0)
    assert r.loss == 0.0
    assert np.all(r.grad == 0.0) and np.all(r.theta == 0.0)
    assert tmpl.shape == (3, 12) and e.shape[0] == 2


def _live_wconf(ctm, cd_max, epoch, e_max):
    """Eq. 15-16 on the template terms of the perturbed grids, with cd_max held
    at the reference forward's value (Eq. 17 detaches it)."""
    delta = 1.0 - np.sqrt(epoch / e_max)
    return np.cumprod((1.0 + np.maximum(0.0, np.asarray(ctm) - cd_max)) ** -delta)


def _frozen_loss(seq, res, theta, ref, hp, epoch):
    """Loss of the step as a function of the grid values with the neighbour
    assignment and cd_max held at ``ref``'s values; the confidence weights
    follow the template terms (Eq. 15)."""
    pts = seq.points
    t_count = pts.shape[0] - 1
    ls = hp.scale(len(res))
    xs = [seq.template.astype(np.float64)]
    for t in range(t_count):
        xs.append(W.warp(theta[t], res, xs[t], ls))
    cpt, ctm = [], []
    for t in range(t_count):
        ph = W.warp(theta[t], res, pts[t], ls)
        tgt = pts[t + 1]
        cpt.append(C.direction_loss(ph, tgt, ref.nn["pt_ab"][t], hp.alpha) +
                   C.direction_loss(tgt, ph, ref.nn["pt_ba"][t], hp.alpha))
        ctm.append(C.direction_loss(xs[t + 1], tgt, ref.nn["tm_ab"][t], hp.alpha) +
                   C.direction_loss(tgt, xs[t + 1], ref.nn["tm_ba"][t], hp.alpha))
    w = _live_wconf(ctm, ref.cd_max, epoch, hp.e_max)
    tot = float(np.sum(w * np.array(ctm) + np.array(cpt)))
    return tot / t_count + S.isometry(np.stack(xs), seq.edges, hp.w_iso)[0]


def test_step_gradient_finite_difference():
    # the full reverse sweep (Chamfer adjoints, isometry, template chain and
    # grid scatter) against central differences of the assembled loss
    seq = _tiny_sequence(frames=4, n=40, subdiv=1, seed=5)
    res = (1, 2, 4)
    hp = S.Hyper(e_max=10)
    rng = np.random.default_rng(6)
    tot = 3 * sum(r ** 3 for r in res)
    theta = rng.normal(0, 0.02, (3, tot))
    z = np.zeros_like(theta)
    ref = S.step(seq.points, seq.template, seq.edges, res, theta, z, z, epoch=2, hp=hp,
                 phat32=None, xhat32=None)
    # the oracle evaluates losses on float32-rounded positions; the frozen
    # loss here is float64, so compare with a tolerance above that rounding
    h = 1e-5
    for t in range(3):
        for k in rng.choice(tot, 5, replace=False):
            tp, tm = theta.copy(), theta.copy()
            tp[t, k] += h
            tm[t, k] -= h
            fd = (_frozen_loss(seq, res, tp, ref, hp, 2) -
                  _frozen_loss(seq, res, tm, ref, hp, 2)) / (2 * h)
            assert abs(fd - ref.grad[t, k]) <= 2e-4 * max(abs(fd), 1e-3), (t, k, fd, ref.grad[t, k])


def test_step_loss_decreases_on_pair():
    src, tgt = synth.pair_on_sphere(seed=0, n=512)
    pts = np.stack([src, tgt])
    res = (8, 16, 32)
    tot = 3 * sum(r ** 3 for r in res)
    th = np.zeros((1, tot))
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    losses = []
    for e in range(6):
        r = S.step(pts, None, None, res, th, m, v, epoch=e, hp=S.Hyper(e_max=6))
        losses.append(r.loss)
        th, m, v = r.theta, r.m, r.v
    assert losses[-1] < 0.8 * losses[0]


def test_template_step_pieces():
    """X_0 optimised (Eq. 9-10, Sec. 3.6): L gains CD_R(X_0, P_0); its gradient
    by central differences; the mesh preconditioner applied to it; Adam's
    first step moves every coordinate by -mesh_lr * sign(g) (bias corrections
    cancel); the paper's mesh constants."""
    from oracle import mesh as M
    h = S.Hyper()
    assert h.mesh_lr == GOLD["mesh_lr"]["value"] and h.mesh_lambda == GOLD["mesh_lambda"]["value"]
    seq = synth.deforming_sequence(seed=3, frames=3, n=300, subdiv=1)
    res = (4, 8)
    T = 2
    P = 3 * sum(r ** 3 for r in res)
    z = np.zeros((T, P))
    x0 = seq.template.astype(np.float32)
    base = S.step(seq.points, x0, seq.edges, res, z, z, z, 0, h)
    r = S.step(seq.points, x0, seq.edges, res, z, z, z, 0, h,
               x0_state=(np.zeros(x0.shape), np.zeros(x0.shape)))
    la, lb, _, _ = C.chamfer(x0, seq.points[0])
    assert r.l_mesh == pytest.approx(la + lb, rel=1e-14)
    assert r.loss == pytest.approx(base.loss + r.l_mesh, rel=1e-14)
    np.testing.assert_array_equal(r.theta, base.theta)        # the grids' update is unchanged
    # gradient of L_mesh by central differences (assignment stable at h = 1e-6)
    x64 = x0.astype(np.float64)
    for c, i in ((0, 3), (1, 17), (2, 40)):
        e = np.zeros_like(x64)
        e[c, i] = 1e-6
        lp = sum(C.chamfer(x64 + e, seq.points[0])[:2])
        lm = sum(C.chamfer(x64 - e, seq.points[0])[:2])
        assert r.g_x0[c, i] == pytest.approx((lp - lm) / 2e-6, rel=1e-5, abs=1e-9)
    np.testing.assert_allclose(r.pg_x0, M.precondition(x0.shape[1], seq.edges, 16.0, r.g_x0),
                               rtol=0, atol=1e-15)
    step = x64 - r.x0
    expect = h.mesh_lr * r.pg_x0 / (np.abs(r.pg_x0) + h.eps)
    np.testing.assert_allclose(step, expect, rtol=1e-9, atol=1e-15)


def _frozen_two_way(seq, res, theta, kr, k, hp, epoch):
    """Loss of a step propagated both ways from keyframe k, as a function of
    the grid values (chain order: backward chain, then forward chain), with
    the assignments and cd_max held at ``kr``'s values and the confidence
    weights following each chain's template terms; 1/T and the isometry
    normalisation use the total T = F - 1."""
    pts = seq.points
    f = pts.shape[0]
    T = f - 1
    e = seq.edges.shape[1]
    ls = hp.scale(len(res))
    tot, iso, t0 = 0.0, 0.0, 0
    for c, fr in enumerate((list(range(k, -1, -1)), list(range(k, f)))):
        r = kr.branches[c]
        if r is None:
            continue
        xs = [seq.template.astype(np.float64)]
        for b in range(len(fr) - 1):
            xs.append(W.warp(theta[t0 + b], res, xs[b], ls))
        cpt, ctm = [], []
        for b in range(len(fr) - 1):
            ph = W.warp(theta[t0 + b], res, pts[fr[b]], ls)
            tgt = pts[fr[b + 1]]
            cpt.append(C.direction_loss(ph, tgt, r.nn["pt_ab"][b], hp.alpha) +
                       C.direction_loss(tgt, ph, r.nn["pt_ba"][b], hp.alpha))
            ctm.append(C.direction_loss(xs[b + 1], tgt, r.nn["tm_ab"][b], hp.alpha) +
                       C.direction_loss(tgt, xs[b + 1], r.nn["tm_ba"][b], hp.alpha))
            i, j = seq.edges
            l1 = np.linalg.norm(xs[b + 1][:, i] - xs[b + 1][:, j], axis=0)
            l0 = np.linalg.norm(xs[b][:, i] - xs[b][:, j], axis=0)
            iso += np.sum(np.abs(l1 - l0))
        w = _live_wconf(ctm, kr.cd_max, epoch, hp.e_max)
        tot += float(np.sum(w * np.array(ctm) + np.array(cpt)))
        t0 += len(fr) - 1
    return tot / T + hp.w_iso * iso / (T * e)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_two_way_step_gradient_and_coupling(k):
    """Reverse-time propagation (Sec. 3.3, end) from keyframe k of 4 frames:
    the gradient of both chains' grids by central differences of the whole
    loss; cd_max is the maximum point term over both chains; each chain's
    confidence weights are the products outward from the keyframe."""
    seq = _tiny_sequence(frames=4, n=40, subdiv=1, seed=8)
    res = (1, 2, 4)
    hp = S.Hyper(e_max=10)
    rng = np.random.default_rng(9)
    tot = 3 * sum(r ** 3 for r in res)
    theta = rng.normal(0, 0.02, (3, tot))
    z = np.zeros_like(theta)
    kr = S.step_keyframe(seq.points, seq.template, seq.edges, res, theta, z, z, 2, k, hp)
    pts = [kr.branches[c].cd_pt.sum(axis=1) for c in (0, 1) if kr.branches[c] is not None]
    assert kr.cd_max == max(float(np.max(p)) for p in pts)
    delta = 1.0 - np.sqrt(2 / 10)
    for r in kr.branches:
        if r is None:
            continue
        tm = r.cd_tm.sum(axis=1)
        w = np.cumprod((1.0 + np.maximum(0.0, tm - kr.cd_max)) ** -delta)
        np.testing.assert_allclose(r.w_conf, w, rtol=1e-14)
    grads = np.concatenate([r.grad for r in kr.branches if r is not None])
    h = 1e-5
    for t in range(3):
        for q in rng.choice(tot, 4, replace=False):
            tp, tq = theta.copy(), theta.copy()
            tp[t, q] += h
            tq[t, q] -= h
            fd = (_frozen_two_way(seq, res, tp, kr, k, hp, 2) -
                  _frozen_two_way(seq, res, tq, kr, k, hp, 2)) / (2 * h)
            assert abs(fd - grads[t, q]) <= 2e-4 * max(abs(fd), 1e-3), (t, q, fd, grads[t, q])


def test_two_way_ends_reduce_to_one_chain():
    seq = _tiny_sequence(frames=4, n=40, subdiv=1, seed=10)
    res = (2, 4)
    hp = S.Hyper(e_max=10)
    theta = np.random.default_rng(11).normal(0, 0.02, (3, 3 * (8 + 64)))
    z = np.zeros_like(theta)
    fwd = S.step(seq.points, seq.template, seq.edges, res, theta, z, z, 1, hp)
    k0 = S.step_keyframe(seq.points, seq.template, seq.edges, res, theta, z, z, 1, 0, hp)
    assert k0.branches[0] is None and k0.loss == fwd.loss
    np.testing.assert_array_equal(k0.theta, fwd.theta)
    rev = S.step(seq.points[::-1], seq.template, seq.edges, res, theta, z, z, 1, hp)
    k3 = S.step_keyframe(seq.points, seq.template, seq.edges, res, theta, z, z, 1, 3, hp)
    assert k3.branches[1] is None and k3.loss == rev.loss
    np.testing.assert_array_equal(k3.theta, rev.theta)


def _frozen_loss6(seq, res, theta, ref, hp, epoch):
    """As _frozen_loss for the six-channel cells (x' = R(z^) x + t^)."""
    from oracle import cayley as CY
    pts = seq.points
    t_count = pts.shape[0] - 1
    ls = hp.scale(len(res))
    xs = [seq.template.astype(np.float64)]
    for t in range(t_count):
        xs.append(CY.warp6(theta[t], res, xs[t], ls))
    cpt, ctm = [], []
    for t in range(t_count):
        ph = CY.warp6(theta[t], res, pts[t], ls)
        tgt = pts[t + 1]
        cpt.append(C.direction_loss(ph, tgt, ref.nn["pt_ab"][t], hp.alpha) +
                   C.direction_loss(tgt, ph, ref.nn["pt_ba"][t], hp.alpha))
        ctm.append(C.direction_loss(xs[t + 1], tgt, ref.nn["tm_ab"][t], hp.alpha) +
                   C.direction_loss(tgt, xs[t + 1], ref.nn["tm_ba"][t], hp.alpha))
    w = _live_wconf(ctm, ref.cd_max, epoch, hp.e_max)
    tot = float(np.sum(w * np.array(ctm) + np.array(cpt)))
    return tot / t_count + S.isometry(np.stack(xs), seq.edges, hp.w_iso)[0]


def test_step_six_channel_gradient_finite_difference():
    """The paper's cells (Eq. 4-7) in the full step: the reverse sweep through
    the rotation-aware adjoints against central differences of the loss, on
    rotation (z) and translation (t) channels alike; the preconditioner and
    Adam treat the six channels of a level alike."""
    from oracle import precond as PC
    seq = _tiny_sequence(frames=3, n=40, subdiv=1, seed=21)
    res = (1, 2, 4)
    hp = S.Hyper(e_max=10)
    rng = np.random.default_rng(22)
    tot = 6 * sum(r ** 3 for r in res)
    theta = rng.normal(0, 0.05, (2, tot))
    z = np.zeros_like(theta)
    ref = S.step(seq.points, seq.template, seq.edges, res, theta, z, z, epoch=1, hp=hp,
                 channels=6)
    h = 1e-5
    for t in range(2):
        for k in rng.choice(tot, 6, replace=False):
            tp, tm = theta.copy(), theta.copy()
            tp[t, k] += h
            tm[t, k] -= h
            fd = (_frozen_loss6(seq, res, tp, ref, hp, 1) -
                  _frozen_loss6(seq, res, tm, ref, hp, 1)) / (2 * h)
            assert abs(fd - ref.grad[t, k]) <= 2e-4 * max(abs(fd), 1e-3), (t, k, fd, ref.grad[t, k])
    # the preconditioner acts on each of the six channels of a level as on the three
    lams = hp.schedule(len(res))[1]
    off = 0
    for r, lam in zip(res, lams):
        blk = ref.grad[0][off:off + 6 * r ** 3].reshape(6, r ** 3)
        np.testing.assert_allclose(ref.pgrad[0][off:off + 6 * r ** 3].reshape(6, -1),
                                   PC.apply_dct(blk, r, lam), atol=1e-15)
        off += 6 * r ** 3


# ---------------------------------------------------------------------------
# The assembled loss against values fixed by hand (Eq. 9, 11-18).
#
# One level of 2^3 cells holding the affine field D(x) = k x (values k times
# the cell centres +-0.5) moves every point inside [-0.5, 0.5]^3 to (1 + k) x
# exactly (trilinear interpolation reproduces affine fields).  The template is
# two vertices (-+1/8, 0, 0) joined by one edge; frame t holds the chain's
# vertices shifted by (0, d_t, 0).  All coordinates are dyadic, so float32
# rounding is exact, and each nearest neighbour is the vertex's own partner.
# Then every Chamfer term is a closed form:
#   CD_R(X_t, P_t)  = 2 d_t^2 e^{-alpha d_t^2},
#   CD_R(P^_t, P_t) = 2 s_t e^{-alpha s_t},  s_t = (d_t - (1 + k_t) d_{t-1})^2,
# and the edge length of frame t is 2/8 times the product of the (1 + k).

def _affine_level(k):
    c = np.array([-0.5, 0.5])
    g = np.zeros((3, 2, 2, 2))
    g[0] = k * c[None, None, :]           # x fastest
    g[1] = k * c[None, :, None]
    g[2] = k * c[:, None, None]
    return g.reshape(-1)


def _two_vertex_frames(scales, offsets):
    x0 = np.array([[-0.125, 0.125], [0.0, 0.0], [0.0, 0.0]])
    return [s * x0 + np.array([[0.0], [d], [0.0]]) for s, d in zip(scales, offsets)], x0


def _cd(s, alpha=5.56):
    return 2.0 * s * np.exp(-alpha * s)


def test_step_loss_hand_value():
    """L of one step (Eq. 9, 14-18) on the two-vertex geometry: T = 2,
    k = (1/4, -1/8), d = (1/4, 1/4, 5/16), epoch 0 of 50 (delta = 1).  Both
    template terms exceed cd_max, so w_conf < 1; a loss that drops w_conf, the
    1/T of Eq. 14 or 18, or the weight 250 misses the hand value."""
    ks, ds = (0.25, -0.125), (0.25, 0.25, 0.3125)
    sig = [1.0, 1.25, 1.25 * 0.875]
    frames, x0 = _two_vertex_frames(sig, ds)
    pts = np.stack(frames).astype(np.float32)
    theta = np.stack([_affine_level(k) for k in ks])
    z = np.zeros_like(theta)
    edges = np.array([[0], [1]], np.int32)
    r = S.step(pts, x0.astype(np.float32), edges, (2,), theta, z, z, 0, S.Hyper(e_max=50))
    # the hand values
    ctm = [_cd(ds[1] ** 2), _cd(ds[2] ** 2)]                      # 2 d^2 e^{-alpha d^2}
    cpt = [_cd((ds[1] - 1.25 * ds[0]) ** 2), _cd((ds[2] - 0.875 * ds[1]) ** 2)]
    cd_max = max(cpt)
    w1 = 1.0 / (1.0 + ctm[0] - cd_max)
    w2 = w1 / (1.0 + ctm[1] - cd_max)
    lens = [0.25 * s for s in sig]
    l_iso = (abs(lens[1] - lens[0]) + abs(lens[2] - lens[1])) / (2 * 1)
    expect = 0.5 * (w1 * ctm[0] + cpt[0] + w2 * ctm[1] + cpt[1]) + 250.0 * l_iso
    np.testing.assert_allclose(r.cd_tm.sum(axis=1), ctm, rtol=1e-14)
    np.testing.assert_allclose(r.cd_pt.sum(axis=1), cpt, rtol=1e-14)
    assert r.cd_max == pytest.approx(cd_max, rel=1e-14)
    np.testing.assert_allclose(r.w_conf, [w1, w2], rtol=1e-14)
    assert w2 < 0.9                                     # the weights matter
    assert r.l_iso == pytest.approx(250.0 * l_iso, rel=1e-14)
    assert r.loss == pytest.approx(expect, rel=1e-14)
    # the template terms' weights in the gradient (Eq. 15 differentiated):
    # dL_T/dCD_1 = w1 - w1 (w1 c1 + w2 c2) / ... by the product rule, by hand
    g1 = w1 - (w1 * ctm[0] + w2 * ctm[1]) / (1.0 + ctm[0] - cd_max)
    g2 = w2 - w2 * ctm[1] / (1.0 + ctm[1] - cd_max)
    np.testing.assert_allclose(r.tm_weight, [g1, g2], rtol=1e-13)


def test_keyframe_loss_hand_value():
    """The same geometry propagated both ways from keyframe 1 of 3 frames:
    the backward grid scales X_0 by 5/4 onto frame 0, the forward one by 7/8
    onto frame 2.  1/T uses the total T = 2, cd_max spans both chains, each
    chain's confidence product has one factor."""
    kb, kf = 0.25, -0.125
    d0, d1, d2 = 0.3125, 0.25, 0.1875
    frames, x0 = _two_vertex_frames((1.0 + kb, 1.0, 1.0 + kf), (d0, d1, d2))
    pts = np.stack(frames).astype(np.float32)
    theta = np.stack([_affine_level(kb), _affine_level(kf)])
    z = np.zeros_like(theta)
    edges = np.array([[0], [1]], np.int32)
    out = S.step_keyframe(pts, x0.astype(np.float32), edges, (2,), theta, z, z, 0, 1,
                          S.Hyper(e_max=50))
    ctm_b, ctm_f = _cd(d0 ** 2), _cd(d2 ** 2)
    cpt_b, cpt_f = _cd((d0 - (1 + kb) * d1) ** 2), _cd((d2 - (1 + kf) * d1) ** 2)
    cd_max = max(cpt_b, cpt_f)
    wb = 1.0 / (1.0 + max(0.0, ctm_b - cd_max))
    wf = 1.0 / (1.0 + max(0.0, ctm_f - cd_max))
    l_iso = (abs(0.25 * (1 + kb) - 0.25) + abs(0.25 * (1 + kf) - 0.25)) / 2
    expect = 0.5 * (wb * ctm_b + cpt_b + wf * ctm_f + cpt_f) + 250.0 * l_iso
    assert out.cd_max == pytest.approx(cd_max, rel=1e-14)
    assert wb < 0.95 and wf < 0.99
    assert out.loss == pytest.approx(expect, rel=1e-14)


def test_template_weight_by_differences():
    """template_weight is the derivative of sum_t w_conf(t) c_t (Eq. 15) with
    cd_max constant: central differences of the confidence product itself,
    terms above and below cd_max, several epochs."""
    rng = np.random.default_rng(30)
    c = rng.uniform(0.01, 0.3, 7)
    cd_max = 0.12
    for epoch in (0, 3, 9):
        w, _, delta = S.confidence(c, [cd_max], epoch, 10)
        g = S.template_weight(c, w, cd_max, delta)
        for tau in range(7):
            if abs(c[tau] - cd_max) < 1e-4:
                continue
            h = 1e-6
            cp, cm = c.copy(), c.copy()
            cp[tau] += h
            cm[tau] -= h
            fp = np.sum(S.confidence(cp, [cd_max], epoch, 10)[0] * cp)
            fm = np.sum(S.confidence(cm, [cd_max], epoch, 10)[0] * cm)
            assert g[tau] == pytest.approx((fp - fm) / (2 * h), rel=1e-7, abs=1e-10)


def test_step_gradient_finite_difference_confidence_active():
    """A template far from the points (scaled by 1.4): its Chamfer terms
    exceed cd_max, the confidence weights fall below 1 and their own
    derivative (Eq. 15 through later frames) is a material part of the grid
    gradient; central differences of the loss with live weights."""
    seq = _tiny_sequence(frames=4, n=40, subdiv=1, seed=5)
    seq.template[:] = (1.4 * seq.template).astype(np.float32)
    res = (1, 2, 4)
    hp = S.Hyper(e_max=10)
    rng = np.random.default_rng(7)
    tot = 3 * sum(r ** 3 for r in res)
    theta = rng.normal(0, 0.02, (3, tot))
    z = np.zeros_like(theta)
    ref = S.step(seq.points, seq.template, seq.edges, res, theta, z, z, epoch=1, hp=hp)
    assert np.all(ref.cd_tm.sum(axis=1) > ref.cd_max) and ref.w_conf[-1] < 0.95
    assert np.max(np.abs(ref.tm_weight - ref.w_conf)) > 0.1
    h = 1e-5
    for t in range(3):
        for k in rng.choice(tot, 5, replace=False):
            tp, tm = theta.copy(), theta.copy()
            tp[t, k] += h
            tm[t, k] -= h
            fd = (_frozen_loss(seq, res, tp, ref, hp, 1) -
                  _frozen_loss(seq, res, tm, ref, hp, 1)) / (2 * h)
            assert abs(fd - ref.grad[t, k]) <= 2e-4 * max(abs(fd), 1e-3), (t, k, fd, ref.grad[t, k])
