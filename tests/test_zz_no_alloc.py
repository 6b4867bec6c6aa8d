"""pdg_chamfer_noalloc (the Chamfer of Eq. 11-13 on the library's fixed
device scratch) against pdg_chamfer with a caller workspace: the same
indices, losses and gradient, bit for bit, on two calls in a row whose second
input is smaller than the first (the scratch keeps the first call's contents),
in both neighbour modes."""
import numpy as np
import pytest
import torch

from paper_2509_18097_amd import _lib as L
from _gpu import dev, require_gpu

pytestmark = pytest.mark.gpu


def _cloud(seed, n):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (3, n)).astype(np.float32)


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_noalloc_equals_workspace_chamfer_twice(mode):
    require_gpu()
    w = dev(np.array([0.7, 1.3]))
    for call, (n, m) in enumerate(((20_000, 17_001), (3_001, 5_000))):
        print(f"no-alloc chamfer mode={mode} call={call} n={n} m={m}", flush=True)
        a = dev(_cloud(10 + call, n))
        b = dev(_cloud(20 + call, m))
        got = L.chamfer_noalloc(a, b, 5.56, mode, dir_weight=w, need_grad=True)
        ref = L.chamfer(a, b, 5.56, mode, dir_weight=w, need_grad=True)
        torch.cuda.synchronize()
        for g, r, what in zip(got, ref, ("loss", "nn_a", "nn_b", "ga")):
            assert torch.equal(g, r), (mode, call, what)
        assert torch.all(got[1] >= 0) and torch.all(got[1] < m)


def test_noalloc_without_gradient_and_repeated_small_call():
    require_gpu()
    a = dev(_cloud(1, 1))
    b = dev(_cloud(2, 1000))
    for _ in range(2):
        loss, nn_a, nn_b, ga = L.chamfer_noalloc(a, b, 5.56, "fp32")
        ref = L.chamfer(a, b, 5.56, "fp32")
        torch.cuda.synchronize()
        assert ga is None
        assert torch.equal(loss, ref[0]) and torch.equal(nn_a, ref[1]) and torch.equal(nn_b, ref[2])
        assert torch.all(nn_b == 0)
