"""Helpers shared by the GPU tests (device transfers and tolerances)."""
import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_rel(got, ref, tol=1e-5, what=""):
    """Norm-relative and max-relative agreement: ||d|| <= tol ||ref|| and
    max|d| <= tol max|ref| (element-relative is meaningless near zero)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = got - ref
    nr = np.linalg.norm(ref)
    mr = np.max(np.abs(ref)) if ref.size else 0.0
    assert np.linalg.norm(d) <= tol * nr + 1e-30, f"{what}: ||d||/||ref|| = {np.linalg.norm(d) / max(nr, 1e-300):.3e}"
    assert np.max(np.abs(d)) <= tol * mr + 1e-30, f"{what}: max|d|/max|ref| = {np.max(np.abs(d)) / max(mr, 1e-300):.3e}"
