"""GPU parity of reverse-time propagation (Sec. 3.3, end): a sequence whose
initial mesh sits at frame k is one problem with a backward chain k -> .. -> 0
and a forward chain k -> .. -> F-1; each chain's stages are compared with the
oracle's two-way step on the GPU's own float32 inputs (indices bit for bit,
losses, confidence weights, shared cd_max, gradients, Adam)."""
import numpy as np
import pytest
import torch

import synth
from oracle import prune as PR
from oracle import sequence as S
from paper_2509_18097_amd import _lib as L
from paper_2509_18097_amd.problem import HyperParams, Problem
from _gpu import assert_rel, dev, host, require_gpu

pytestmark = pytest.mark.gpu

RES = (4, 8, 16)


def _setup(seed=12, frames=5, n=700, subdiv=2):
    seq = synth.deforming_sequence(seed=seed, frames=frames, n=n, subdiv=subdiv)
    theta0 = np.random.default_rng(seed).normal(0, 0.01, (frames - 1, L.grid_size(RES))).astype(np.float32)
    return seq, theta0


def _problem(seq, theta0, k, mode="fp32", **kw):
    return Problem(dev(seq.points), RES, template=dev(seq.template), edges=dev(seq.edges),
                   hp=HyperParams(e_max=10), params=dev(theta0), chamfer_mode=mode, keyframe=k,
                   **kw)


@pytest.mark.parametrize("k,mode", [(2, "fp32"), (2, "bf16"), (1, "fp32"), (4, "fp32")])
def test_two_way_step_matches_oracle(k, mode):
    require_gpu()
    seq, theta0 = _setup()
    prob = _problem(seq, theta0, k, mode, precond="dct")
    prob.step(1)
    prob.stage("precond")          # the preconditioned gradient of every level
    torch.cuda.synchronize()
    chains = [prob.branch(0), prob.branch(1)]
    assert (chains[0] is None) == (k == 0) and (chains[1] is None) == (k == 4)
    ov = [None if ch is None else
          dict(phat32=host(ch.buffer("phat")), xhat32=host(ch.buffer("xhat")),
               grad_override=host(ch.buffer("grad")), pgrad_override=host(ch.buffer("pgrad")))
          for ch in chains]
    z = np.zeros_like(theta0, dtype=np.float64)
    r = S.step_keyframe(seq.points, seq.template, seq.edges, RES, theta0, z, z, 1, k,
                        S.Hyper(e_max=10), overrides=ov, workers=4)
    for c, ch in enumerate(chains):
        if ch is None:
            assert r.branches[c] is None
            continue
        rb = r.branches[c]
        Tc = ch.T
        np.testing.assert_array_equal(host(ch.buffer("xhat"))[0], seq.template)
        nn = {key: host(v) for key, v in ch.nn().items()}
        for key, v in rb.nn.items():
            np.testing.assert_array_equal(nn[key], v, err_msg=f"chain {c} {key}")
        losses = host(ch.buffer("losses"))
        np.testing.assert_allclose(losses[:Tc], rb.cd_pt, rtol=1e-10, atol=0)
        np.testing.assert_allclose(losses[Tc:2 * Tc], rb.cd_tm, rtol=1e-10, atol=0)
        np.testing.assert_allclose(host(ch.buffer("wconf")), rb.w_conf, rtol=1e-12, atol=0)
        assert_rel(host(ch.buffer("grad")), rb.grad, 1e-5, f"chain {c} dL/dG")
        assert_rel(host(ch.buffer("pgrad")), rb.pgrad, 1e-5, f"chain {c} preconditioned")
    terms = prob.terms()
    assert abs(terms["loss"] - r.loss) <= 1e-10 * abs(r.loss)
    assert abs(terms["cd_max"] - r.cd_max) <= 1e-12 * r.cd_max
    eta_max = max(S.Hyper().schedule(len(RES))[0])
    assert np.max(np.abs(host(prob.params) - r.theta)) <= 1e-5 * eta_max


def test_two_way_graph_replay_equals_eager():
    require_gpu()
    seq, theta0 = _setup(seed=13, frames=4, n=500, subdiv=1)
    a = _problem(seq, theta0, 2, "bf16", optimize_template=True)
    b = _problem(seq, theta0, 2, "bf16", optimize_template=True)
    for e in range(3):
        a.step(e)
        b.step(e, use_graph=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(a.params), host(b.params))
        np.testing.assert_array_equal(host(a.template), host(b.template))
        assert a.terms() == b.terms()
    assert a.terms()["l_mesh"] > 0.0


def test_two_way_pruned_masks_in_chain_order():
    require_gpu()
    seq, theta0 = _setup(seed=14, frames=5, n=400, subdiv=1)
    prob = _problem(seq, theta0, 3, precond="cg", prune_halo=1)
    got = host(prob.prune_mask)
    ref = PR.stack_masks(seq.points, RES, halo=1, span=2)
    words = L.prune_mask_words(RES)
    for i, j in enumerate([2, 1, 0, 3]):          # chain order for k = 3 of 5 frames
        bits = np.zeros(words * 32, dtype=bool)
        off = 0
        for mk, r in zip(ref[j], RES):
            bits[off:off + r ** 3] = mk.reshape(-1)
            off += -(-r ** 3 // 32) * 32
        w = (bits.reshape(-1, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(1)
        np.testing.assert_array_equal(got[i].view(np.uint32), w.astype(np.uint32))
    # each chain's step against the oracle's on the kept cells' graphs
    order = [2, 1, 0, 3]
    keep = np.stack([PR.packed_mask(ref[j], RES) for j in order])
    theta_p = np.where(keep, theta0, 0.0).astype(np.float32)
    np.testing.assert_array_equal(host(prob.params), theta_p)
    prob.step(0)
    torch.cuda.synchronize()
    chains = [prob.branch(0), prob.branch(1)]
    ov = [dict(phat32=host(ch.buffer("phat")), xhat32=host(ch.buffer("xhat")),
               grad_override=host(ch.buffer("grad")), pgrad_override=host(ch.buffer("pgrad")),
               masks=[ref[j] for j in js])
          for ch, js in zip(chains, ([2, 1, 0], [3]))]
    z = np.zeros_like(theta_p, dtype=np.float64)
    r = S.step_keyframe(seq.points, seq.template, seq.edges, RES, theta_p, z, z, 0, 3,
                        S.Hyper(e_max=10), overrides=ov, workers=4)
    for c, ch in enumerate(chains):
        rb = r.branches[c]
        assert_rel(host(ch.buffer("grad")), rb.grad, 1e-5, f"chain {c} dL/dG")
        assert_rel(host(ch.buffer("pgrad")), rb.pgrad, 1e-5, f"chain {c} pruned preconditioned")
    assert abs(prob.terms()["loss"] - r.loss) <= 1e-10 * abs(r.loss)
    eta_max = max(S.Hyper().schedule(len(RES))[0])
    params = host(prob.params)
    assert np.max(np.abs(params - r.theta)) <= 1e-5 * eta_max
    assert np.all(params[~keep] == 0.0)


def test_joint_handle_buffers():
    require_gpu()
    seq, theta0 = _setup(seed=15, frames=4, n=300, subdiv=1)
    prob = _problem(seq, theta0, 1)
    prob.step(0)
    with pytest.raises(L.PdgError, match="per chain"):
        prob.buffer("grad")
    assert prob.branch(0).T == 1 and prob.branch(1).T == 2


def test_keyframe_last_frame_optimises_template_with_the_backward_chain():
    """With X_0 at the last frame only the backward chain exists; X_0 is then
    optimised with it (L_mesh against P_k), as the oracle's two-way step does."""
    require_gpu()
    seq, theta0 = _setup(seed=16, frames=4, n=500, subdiv=1)
    k = 3
    prob = _problem(seq, theta0, k, "fp32", precond="dct", optimize_template=True)
    prob.step(0)
    prob.stage("precond")
    torch.cuda.synchronize()
    ch = prob.branch(0)
    assert prob.branch(1) is None and ch.T == 3
    V = seq.template.shape[1]
    ov = [dict(phat32=host(ch.buffer("phat")), xhat32=host(ch.buffer("xhat")),
               grad_override=host(ch.buffer("grad")), pgrad_override=host(ch.buffer("pgrad")),
               gx0_override=host(ch.buffer("gx0")), pgx0_override=host(ch.buffer("pgx0"))), None]
    z = np.zeros_like(theta0, dtype=np.float64)
    r = S.step_keyframe(seq.points, seq.template, seq.edges, RES, theta0, z, z, 0, k,
                        S.Hyper(e_max=10), overrides=ov,
                        x0_state=(np.zeros((3, V)), np.zeros((3, V))))
    rb = r.branches[0]
    nn0 = host(ch.buffer("nn0"))
    np.testing.assert_array_equal(nn0[:V], rb.nn0[0])
    np.testing.assert_array_equal(nn0[V:], rb.nn0[1])
    terms = prob.terms()
    assert abs(terms["l_mesh"] - rb.l_mesh) <= 1e-10 * rb.l_mesh
    assert abs(terms["loss"] - r.loss) <= 1e-10 * abs(r.loss)
    x0 = host(prob.template)
    assert np.all(np.abs(x0 - rb.x0) <= 1e-5 * S.Hyper().mesh_lr + 2.0 ** -23 * np.abs(rb.x0))
