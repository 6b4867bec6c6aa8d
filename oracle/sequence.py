"""Losses and one optimisation step of the method -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's Sec. 3.3-3.6:
* the template chain X_t = warp(G_t, X_{t-1}) (Eq. 8, translation form);
* the point term P^_t = warp(G_t, P_{t-1}) (text after Eq. 14);
* L_transform = 1/T sum_t [ w_conf(t) CD_R(X_t, P_t) + CD_R(P^_t, P_t) ] (Eq. 14);
* w_conf(t) = prod_{tau <= t} (1 + max(0, CD_R(X_tau, P_tau) - cd_max))^{-delta}
  with delta = 1 - sqrt(e / e_max) (Eq. 15-16) and
  cd_max = max_t CD_R(sg(P^_t), P_t) (Eq. 17);
* L_iso = 1/(T |E|) sum_t sum_(i,j) | |x_i,t - x_j,t| - |x_i,t-1 - x_j,t-1| | (Eq. 18);
* L = L_transform + w_iso L_iso, w_iso = 250 (Eq. 9), plus L_mesh =
  CD_R(X_0, P_0) (Eq. 10) when X_0 is optimised (``x0_state``);
* gradients preconditioned per level by (I + lambda_l L_l)^{-2} (Eq. 3) and
  applied by Adam with a per-level learning rate (Sec. 3.6).

Readings:
* Frame 0 is the keyframe; T = F - 1 transitions, grid G_t maps frame t-1 to t.
* Eq. 14 is read as 1/T sum_t [w_conf(t) CD(X, P) + CD(P^, P)].
* w_conf is differentiated with respect to the template terms
  CD_R(X_tau, P_tau) it is built from: Eq. 17 puts the stop-gradient on the
  point terms inside cd_max only, which would be needless if w_conf carried no
  gradient.  cd_max itself is constant for the gradient.  tau runs from 1 to t
  inclusive; e is the 0-based epoch and e_max the number of epochs; the
  derivative of max(0, x) at x = 0 is taken as 0.
* cd_max is taken from the current iteration's forward pass.
* Isometry: sign(0) = 0; a zero-length edge contributes no gradient; X_0 is
  fixed.
* "+10% / +50% per finer level" (Sec. 3.6) compounds:
  eta_l = 5e-3 * 1.1^l, lambda_l = 0.25 * 1.5^l for the 0-based level l.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import adam as _adam
from . import cayley as _cy
from . import chamfer as _ch
from . import mesh as _mesh
from . import precond as _pc
from . import prune as _pr
from . import warp as _wp


@dataclass
class Hyper:
    alpha: float = 5.56           # Eq. 13
    w_iso: float = 250.0          # Eq. 9
    eta0: float = 5e-3            # Sec. 3.6
    eta_growth: float = 1.1
    lam0: float = 0.25
    lam_growth: float = 1.5
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    e_max: int = 50
    level_scale: float | None = None     # 1/L (Eq. 1) when None
    mesh_lambda: float = 16.0     # Sec. 3.6: X_0's preconditioner weight
    mesh_lr: float = 1e-4         # Sec. 3.6: X_0's learning rate

    def schedule(self, levels: int):
        etas = [self.eta0 * self.eta_growth ** l for l in range(levels)]
        lams = [self.lam0 * self.lam_growth ** l for l in range(levels)]
        return etas, lams

    def scale(self, levels: int) -> float:
        return 1.0 / levels if self.level_scale is None else float(self.level_scale)


def isometry(xhat: np.ndarray, edges: np.ndarray, w_iso: float = 1.0):
    """Eq. 18 and its gradient.  xhat (F, 3, V) with frame 0 the fixed X_0,
    edges (2, E).  Returns (L_iso, grad (F, 3, V)) of w_iso * L_iso."""
    x = np.asarray(xhat, np.float64)
    f = x.shape[0]
    t_count = f - 1
    i, j = np.asarray(edges[0], np.int64), np.asarray(edges[1], np.int64)
    e = i.shape[0]
    d = x[:, :, i] - x[:, :, j]                   # (F, 3, E)
    ln = np.sqrt(np.sum(d * d, axis=1))           # (F, E)
    diff = ln[1:] - ln[:-1]                       # (T, E)
    loss = float(np.sum(np.abs(diff)) / (t_count * e))
    sig = np.sign(diff)                           # sign(0) = 0
    coef = w_iso / (t_count * e)
    # frame t gets +sig_t (as the later slice) and -sig_{t+1} (as the earlier)
    s = np.zeros((f, e))
    s[1:] += sig
    s[:-1] -= sig
    u = np.divide(d, ln[:, None, :], out=np.zeros_like(d), where=ln[:, None, :] > 0)
    contrib = coef * s[:, None, :] * u            # (F, 3, E)
    g = np.zeros_like(x)
    for c in range(3):
        for t in range(f):
            np.add.at(g[t, c], i, contrib[t, c])
            np.add.at(g[t, c], j, -contrib[t, c])
    return w_iso * loss, g


def confidence(cd_tm, cd_pt, epoch: int, e_max: int, cd_max: float | None = None):
    """Eq. 15-17.  Returns (w_conf (T,), cd_max, delta); cd_max, when given,
    replaces the maximum of cd_pt (a sequence of several chains shares it)."""
    cd_tm = np.asarray(cd_tm, np.float64)
    cd_max = float(np.max(cd_pt)) if cd_max is None else float(cd_max)
    delta = 1.0 - np.sqrt(epoch / e_max)
    factors = (1.0 / (1.0 + np.maximum(0.0, cd_tm - cd_max))) ** delta
    return np.cumprod(factors), cd_max, float(delta)


def template_weight(cd_tm, w_conf, cd_max: float, delta: float) -> np.ndarray:
    """d/dCD_R(X_tau, P_tau) of sum_t w_conf(t) CD_R(X_t, P_t) (Eq. 14-15),
    with cd_max held constant (Eq. 17): w_conf(tau) from the term itself, plus,
    when CD_R(X_tau, P_tau) > cd_max, the change of every later weight through
    its factor tau,
        - delta / (1 + CD_R(X_tau, P_tau) - cd_max) * sum_{t >= tau} w_conf(t) CD_R(X_t, P_t).
    """
    c = np.asarray(cd_tm, np.float64)
    w = np.asarray(w_conf, np.float64)
    later = np.cumsum((w * c)[::-1])[::-1]         # sum over t >= tau
    active = c - cd_max > 0.0
    dlog = np.where(active, -delta / (1.0 + np.where(active, c - cd_max, 0.0)), 0.0)
    return w + dlog * later


@dataclass
class StepResult:
    phat: np.ndarray                  # (T, 3, N) float64 warped input points
    xhat: np.ndarray | None           # (F, 3, V) float64 template chain
    nn: dict = field(default_factory=dict)       # 'pt_ab', 'pt_ba', 'tm_ab', 'tm_ba': (T, ...) int64
    cd_pt: np.ndarray = None          # (T, 2) per direction
    cd_tm: np.ndarray = None          # (T, 2)
    cd_max: float = 0.0
    w_conf: np.ndarray = None
    tm_weight: np.ndarray = None      # (T,) dL_transform/dCD_R(X_t, P_t) times T
    l_iso: float = 0.0
    loss: float = 0.0
    grad: np.ndarray = None           # (T, P) raw packed grid gradient
    pgrad: np.ndarray = None          # (T, P) preconditioned
    theta: np.ndarray = None          # (T, P) after Adam
    m: np.ndarray = None
    v: np.ndarray = None
    g_phat: np.ndarray = None         # (T, 3, N) dL/dP^_t
    g_xhat: np.ndarray = None         # (T, 3, V) dL/dX_t (direct terms, frames 1..T)
    # optimisation of X_0 (Eq. 9-10, Sec. 3.6), when asked for
    l_mesh: float = 0.0
    nn0: tuple = None                 # (nn of X_0 in P_0, nn of P_0 in X_0)
    g_x0: np.ndarray = None           # (3, V) dL_mesh/dX_0
    pg_x0: np.ndarray = None          # (3, V) (I + mesh_lambda L)^-2 g_x0
    x0: np.ndarray = None             # (3, V) X_0 after Adam
    x0_m: np.ndarray = None
    x0_v: np.ndarray = None


def step(points, template, edges, res, theta, m, v, epoch: int, hp: Hyper = Hyper(),
         phat32=None, xhat32=None, workers: int = 1, precond_method: str = "dct",
         grad_override=None, pgrad_override=None, masks=None, x0_state=None,
         gx0_override=None, pgx0_override=None, t_norm: int | None = None,
         cd_max: float | None = None, channels: int = 3) -> StepResult:
    """One iteration: warp, Chamfer + isometry losses, gradient, preconditioner, Adam.

    points (F, 3, N) float32; template (3, V) float32 or None; edges (2, E);
    theta, m, v (T, P) packed per-transition grid values.

    ``phat32`` / ``xhat32`` give float32 warped positions on which to take the
    nearest-neighbour decisions (so that another implementation's indices can
    be compared on identical inputs); by default the oracle's own float64
    positions are rounded to float32.  ``grad_override`` / ``pgrad_override``
    replace the raw / preconditioned gradient fed to the following stage.
    ``masks`` ([t][level] boolean [r, r, r], see ``prune``) prunes the grids:
    the preconditioner acts on the kept cells only and is zero elsewhere.
    ``x0_state`` = (m, v), the Adam moments of X_0, optimises X_0 as well:
    L gains L_mesh = CD_R(X_0, P_0) (Eq. 9-10), whose gradient alone moves X_0
    (reading: the mesh follows the keyframe's points; the chain's terms are
    not differentiated with respect to X_0), preconditioned by
    (I + mesh_lambda L)^-2 with the mesh Laplacian and applied by Adam with
    mesh_lr (Sec. 3.6).  ``gx0_override`` / ``pgx0_override`` replace the raw /
    preconditioned X_0 gradient fed to the next stage.
    ``t_norm`` / ``cd_max`` (one chain of a sequence propagated both ways from
    its keyframe, see ``step_keyframe``) replace T in the 1/T of Eq. 14 and
    Eq. 18 and the chain's own cd_max of Eq. 17.
    ``channels`` = 6 takes the paper's own cells [z; t] (Eq. 4-7, ``cayley``):
    every warp is x' = R(z^) x + t^, the adjoints are the rotation-aware ones,
    and the preconditioner and Adam treat all six channels of a level alike.
    """
    points = np.asarray(points)
    f = points.shape[0]
    t_count = f - 1
    levels = len(res)
    ls = hp.scale(levels)
    etas, lams = hp.schedule(levels)
    theta = np.asarray(theta, np.float64)
    has_tm = template is not None and np.asarray(template).shape[1] > 0
    tn = t_count if t_norm is None else int(t_norm)
    if channels == 6:
        def warp_fn(th, x):
            return _cy.warp6(th, res, x, ls)

        def grid_adj(th, x, g):
            return _cy.grid_adjoint6(th, res, x, g, ls)

        def pos_adj(th, x, g):
            return _cy.position_adjoint6(th, res, x, g, ls)
    else:
        def warp_fn(th, x):
            return _wp.warp(th, res, x, ls)

        def grid_adj(th, x, g):
            return _wp.grid_adjoint(res, x, g, ls)

        def pos_adj(th, x, g):
            return _wp.position_adjoint(th, res, x, g, ls)

    phat = np.stack([warp_fn(theta[t], points[t]) for t in range(t_count)])
    xhat = None
    if has_tm:
        xs = [np.asarray(template, np.float64)]
        for t in range(t_count):
            src = xs[t] if xhat32 is None else np.asarray(xhat32[t], np.float64)
            xs.append(warp_fn(theta[t], src))
        xhat = np.stack(xs)
    p_nn = phat.astype(np.float32) if phat32 is None else np.asarray(phat32, np.float32)
    x_nn = None
    if has_tm:
        x_nn = xhat.astype(np.float32) if xhat32 is None else np.asarray(xhat32, np.float32)

    r = StepResult(phat=phat, xhat=xhat)
    cd_pt = np.zeros((t_count, 2))
    cd_tm = np.zeros((t_count, 2))
    nn = {k: [] for k in ("pt_ab", "pt_ba", "tm_ab", "tm_ba")}
    for t in range(t_count):
        tgt = points[t + 1]
        a = p_nn[t]
        na = _ch.nn_fp32(a, tgt, workers=workers)
        nb = _ch.nn_fp32(tgt, a, workers=workers)
        nn["pt_ab"].append(na)
        nn["pt_ba"].append(nb)
        cd_pt[t] = (_ch.direction_loss(a, tgt, na, hp.alpha),
                    _ch.direction_loss(tgt, a, nb, hp.alpha))
        if has_tm:
            a = x_nn[t + 1]
            na = _ch.nn_fp32(a, tgt, workers=workers)
            nb = _ch.nn_fp32(tgt, a, workers=workers)
            nn["tm_ab"].append(na)
            nn["tm_ba"].append(nb)
            cd_tm[t] = (_ch.direction_loss(a, tgt, na, hp.alpha),
                        _ch.direction_loss(tgt, a, nb, hp.alpha))
    r.nn = {k: np.stack(vv) for k, vv in nn.items() if vv}
    r.cd_pt, r.cd_tm = cd_pt, cd_tm
    pt = cd_pt.sum(axis=1)
    tm = cd_tm.sum(axis=1)
    if has_tm:
        w_conf, cd_max, delta = confidence(tm, pt, epoch, hp.e_max, cd_max)
        tm_w = template_weight(tm, w_conf, cd_max, delta)
        l_iso, g_iso = isometry(x_nn, edges, hp.w_iso)
        l_iso, g_iso = l_iso * t_count / tn, g_iso * (t_count / tn)
    else:
        w_conf, l_iso, g_iso = np.ones(t_count), 0.0, None
        tm_w = np.ones(t_count)
        cd_max = float(np.max(pt)) if cd_max is None else float(cd_max)
    r.w_conf, r.cd_max, r.l_iso, r.tm_weight = w_conf, cd_max, l_iso, tm_w
    r.loss = float(np.sum(w_conf * tm + pt) / tn + l_iso) if has_tm else float(np.sum(pt) / tn)

    # gradients of the loss with respect to the warped positions
    g_phat = np.stack([_ch.gradient(p_nn[t], points[t + 1], r.nn["pt_ab"][t], r.nn["pt_ba"][t],
                                    hp.alpha, 1.0 / tn, 1.0 / tn)
                       for t in range(t_count)])
    r.g_phat = g_phat
    grad = np.stack([grid_adj(theta[t], points[t], g_phat[t]) for t in range(t_count)])
    if has_tm:
        g_x = np.stack([_ch.gradient(x_nn[t + 1], points[t + 1], r.nn["tm_ab"][t], r.nn["tm_ba"][t],
                                     hp.alpha, tm_w[t] / tn, tm_w[t] / tn)
                        for t in range(t_count)]) + g_iso[1:]
        r.g_xhat = g_x
        chain_pos = x_nn
        lam = g_x[t_count - 1]
        for t in range(t_count - 1, -1, -1):
            grad[t] += grid_adj(theta[t], chain_pos[t], lam)
            if t > 0:
                lam = g_x[t - 1] + pos_adj(theta[t], chain_pos[t], lam)
    r.grad = grad
    g_in = grad if grad_override is None else np.asarray(grad_override, np.float64)
    if masks is None:
        pgrad = np.stack([_pc.apply_levels(g_in[t], res, lams, precond_method, channels)
                          for t in range(t_count)])
    else:
        pgrad = np.stack([_pr.apply_levels_masked(g_in[t], res, lams, masks[t], channels)
                          for t in range(t_count)])
    r.pgrad = pgrad
    p_in = pgrad if pgrad_override is None else np.asarray(pgrad_override, np.float64)
    th, mm, vv = np.empty_like(theta), np.empty_like(theta), np.empty_like(theta)
    off = 0
    for l, rr in enumerate(res):
        sl = slice(off, off + channels * rr ** 3)
        th[:, sl], mm[:, sl], vv[:, sl] = _adam.update(
            theta[:, sl], np.asarray(m)[:, sl], np.asarray(v)[:, sl], p_in[:, sl], etas[l],
            epoch + 1, hp.beta1, hp.beta2, hp.eps)
        off += channels * rr ** 3
    r.theta, r.m, r.v = th, mm, vv
    if x0_state is not None and has_tm:
        x0 = np.asarray(template, np.float32)
        p0 = points[0]
        l_ab, l_ba, na, nb = _ch.chamfer(x0, p0, hp.alpha, workers=workers)
        r.l_mesh = float(l_ab + l_ba)
        r.loss += r.l_mesh
        r.nn0 = (na, nb)
        r.g_x0 = _ch.gradient(x0, p0, na, nb, hp.alpha, 1.0, 1.0)
        g_in = r.g_x0 if gx0_override is None else np.asarray(gx0_override, np.float64)
        r.pg_x0 = _mesh.precondition(x0.shape[1], edges, hp.mesh_lambda, g_in)
        p_in = r.pg_x0 if pgx0_override is None else np.asarray(pgx0_override, np.float64)
        r.x0, r.x0_m, r.x0_v = _adam.update(x0, x0_state[0], x0_state[1], p_in, hp.mesh_lr,
                                            epoch + 1, hp.beta1, hp.beta2, hp.eps)
    return r


@dataclass
class KeyframeResult:
    branches: list                    # [backward, forward] StepResult or None
    loss: float = 0.0
    cd_max: float = 0.0
    theta: np.ndarray = None          # (T, P) chain order: backward, then forward
    m: np.ndarray = None
    v: np.ndarray = None


def chains(frames: int, keyframe: int):
    """Frame order of the two chains leaving keyframe k (Sec. 3.3, end): the
    backward chain k, k-1, .., 0 and the forward chain k, k+1, .., F-1; a
    chain of one frame holds no transition."""
    return list(range(keyframe, -1, -1)), list(range(keyframe, frames))


def step_keyframe(points, template, edges, res, theta, m, v, epoch: int, keyframe: int,
                  hp: Hyper = Hyper(), workers: int = 1, precond_method: str = "dct",
                  overrides=(None, None), x0_state=None) -> KeyframeResult:
    """One iteration of a sequence whose initial mesh X_0 sits at frame k:
    the transformations are propagated backward from k to frame 0 and forward
    from k to frame F-1 (the mechanism of Eq. 8 applied in reverse, Sec. 3.3).

    Readings: the T = F - 1 grids are ordered by chain, the backward chain's
    (frame k - b + 1 -> k - b, b = 1..k) first, then the forward chain's
    (frame k + f - 1 -> k + f); Eq. 14 and 18 normalise by the total T; cd_max
    of Eq. 17 is the maximum over every transition of both chains; the
    confidence products of Eq. 15 run outward from the keyframe along each
    chain; L_mesh (when X_0 is optimised) is counted once, with the forward
    chain (the backward one when k = F - 1).

    overrides: per chain, a dict of ``step``'s float32 overrides (phat32,
    xhat32, grad_override, pgrad_override, gx0_override, pgx0_override).
    """
    points = np.asarray(points)
    f = points.shape[0]
    t_all = f - 1
    order = chains(f, keyframe)
    theta = np.asarray(theta, np.float64)
    m = np.asarray(m, np.float64)
    v = np.asarray(v, np.float64)
    ls = hp.scale(len(res))
    # cd_max over both chains (the point term of every transition, Eq. 17)
    pt_all = []
    t0 = 0
    for c, fr in enumerate(order):
        ov = overrides[c] or {}
        for b in range(len(fr) - 1):
            if ov.get("phat32") is not None:
                a = np.asarray(ov["phat32"][b], np.float32)
            else:
                a = _wp.warp(theta[t0 + b], res, points[fr[b]], ls).astype(np.float32)
            la, lb, _, _ = _ch.chamfer(a, points[fr[b + 1]], hp.alpha, workers=workers)
            pt_all.append(la + lb)
        t0 += len(fr) - 1
    cd_max = float(np.max(pt_all))
    out = KeyframeResult(branches=[None, None], cd_max=cd_max)
    th, mm, vv = np.empty_like(theta), np.empty_like(theta), np.empty_like(theta)
    t0 = 0
    mesh_chain = 1 if len(order[1]) > 1 else 0
    for c, fr in enumerate(order):
        tc = len(fr) - 1
        if tc == 0:
            continue
        sl = slice(t0, t0 + tc)
        r = step(points[fr], template, edges, res, theta[sl], m[sl], v[sl], epoch, hp,
                 workers=workers, precond_method=precond_method, t_norm=t_all, cd_max=cd_max,
                 x0_state=x0_state if c == mesh_chain else None, **(overrides[c] or {}))
        out.branches[c] = r
        out.loss += r.loss
        th[sl], mm[sl], vv[sl] = r.theta, r.m, r.v
        t0 += tc
    out.theta, out.m, out.v = th, mm, vv
    return out
