"""The C-ABI library loads, exports every symbol include/pdg.h declares, and
rejects invalid arguments on the host before touching the GPU."""
import ctypes
import os
import re

import pytest

import conftest
from paper_2509_18097_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pdg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pdg_[a-z_]+)\s*\(", txt)))


def test_library_built():
    assert conftest.BUILD_ERROR is None, conftest.BUILD_ERROR
    assert os.path.exists(L.LIB_PATH)


def test_every_declared_symbol_is_exported_and_bound():
    decl = _declared()
    assert len(decl) >= 15
    h = ctypes.CDLL(L.LIB_PATH)
    for name in decl:
        assert hasattr(h, name), name
        assert name in L.EXPORTS, name


def test_version_and_grid_size():
    lib = L.lib()
    assert lib.pdg_version() >= 100
    d = L.grid_desc((8, 16, 32))
    assert lib.pdg_grid_size(ctypes.byref(d)) == 3 * (8 ** 3 + 16 ** 3 + 32 ** 3)
    bad = L.grid_desc((8,))
    bad.levels = 0
    assert lib.pdg_grid_size(ctypes.byref(bad)) == -1


def test_argument_errors_on_host():
    lib = L.lib()
    d = L.grid_desc((4, 8))
    d.levels = L.MAX_LEVELS + 1
    st = lib.pdg_deform(ctypes.byref(d), None, None, 10, None, None)
    assert st == L.EINVAL and "levels" in L.last_error()
    d = L.grid_desc((4, 8))
    d.channels = 5
    assert lib.pdg_deform(ctypes.byref(d), None, None, 10, None, None) == L.EINVAL
    # six-channel (Cayley) cells: taken by the deform calls, refused elsewhere
    d = L.grid_desc((4, 8), channels=6)
    assert lib.pdg_grid_size(ctypes.byref(d)) == 6 * (4 ** 3 + 8 ** 3)
    assert lib.pdg_deform(ctypes.byref(d), None, None, 10, None, None) == L.EINVAL
    assert "NULL" in L.last_error()
    nb6 = ctypes.c_size_t()
    assert lib.pdg_deform_backward_workspace(ctypes.byref(d), 100, ctypes.byref(nb6)) == L.OK
    # six channels are preconditioned as two three-channel halves
    assert lib.pdg_precondition_workspace(ctypes.byref(d), 1, 0, ctypes.byref(nb6)) == L.OK
    d = L.grid_desc((4, 8))
    assert lib.pdg_deform(ctypes.byref(d), None, None, 10, None, None) == L.EINVAL
    assert "NULL" in L.last_error()
    assert lib.pdg_deform(ctypes.byref(d), None, None, 0, None, None) == L.OK  # empty is a no-op
    nb = ctypes.c_size_t()
    assert lib.pdg_chamfer_workspace(0, 5, 0, ctypes.byref(nb)) == L.EINVAL
    assert lib.pdg_chamfer_workspace(5, 5, 7, ctypes.byref(nb)) == L.EINVAL
    assert lib.pdg_chamfer_workspace(100, 50, 0, ctypes.byref(nb)) == L.OK and nb.value > 0
    lam = (ctypes.c_float * 8)(-1.0, 1.0)
    assert lib.pdg_precondition(ctypes.byref(d), lam, None, 1, 0, 0, 1e-7, None, 0, None) == L.EINVAL
    lam = (ctypes.c_float * 8)(0.25, 0.375)
    assert lib.pdg_precondition(ctypes.byref(d), lam, None, 1, 0, 0, 0.0, None, 0, None) == L.EINVAL
    assert lib.pdg_precondition_workspace(ctypes.byref(d), 2, 0, ctypes.byref(nb)) == L.OK


def test_prune_validation_on_host():
    lib = L.lib()
    d = L.grid_desc((1, 3, 8, 32))
    w = ctypes.c_int64()
    assert lib.pdg_prune_mask_words(ctypes.byref(d), ctypes.byref(w)) == L.OK
    assert w.value == 1 + 1 + 16 + 1024 == L.prune_mask_words((1, 3, 8, 32))
    nb = ctypes.c_size_t()
    assert lib.pdg_prune_workspace(ctypes.byref(d), 3, ctypes.byref(nb)) == L.OK
    assert nb.value >= 2 * 3 * w.value * 4
    # halo out of range, span < 1, NULL mask, too small a workspace: nothing runs
    assert lib.pdg_prune_mask(ctypes.byref(d), 2, 2, None, 0, 17, None, None, None, 0, None) == L.EINVAL
    assert lib.pdg_prune_mask(ctypes.byref(d), 2, 0, None, 0, 3, None, None, None, 0, None) == L.EINVAL
    assert lib.pdg_prune_mask(ctypes.byref(d), 2, 2, None, 0, 3, None, None, None, 0, None) == L.EINVAL
    assert lib.pdg_prune_mask(ctypes.byref(d), 2, 2, None, 0, 3, 256, None, 256, 8, None) == L.ENOMEM
    assert lib.pdg_prune_mask(ctypes.byref(d), 0, 2, None, 0, 3, None, None, None, 0, None) == L.OK
    lam = (ctypes.c_float * 16)(0.25, 0.375, 0.5, 0.75)
    assert lib.pdg_precondition_pruned(ctypes.byref(d), lam, 256, 1, 0, 1e-7, None, None, 0,
                                       None) == L.EINVAL
    assert lib.pdg_precondition_pruned(ctypes.byref(d), lam, 256, 1, 0, 1e-7, 256, 256, 8,
                                       None) == L.ENOMEM
    # masks cover cells: a six-channel descriptor has the same words
    d6 = L.grid_desc((4, 8), channels=6)
    w3, w6 = ctypes.c_int64(), ctypes.c_int64()
    assert lib.pdg_prune_mask_words(ctypes.byref(L.grid_desc((4, 8))), ctypes.byref(w3)) == L.OK
    assert lib.pdg_prune_mask_words(ctypes.byref(d6), ctypes.byref(w6)) == L.OK
    assert w6.value == w3.value == 2 + 16


def test_problem_validation_on_host():
    lib = L.lib()
    pd = L.ProblemDesc()
    pd.frames = 1
    pd.n = 10
    pd.grid = L.grid_desc((4, 8))
    nb = ctypes.c_size_t()
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.EINVAL
    assert "frames" in L.last_error()
    pd.frames = 3
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.EINVAL  # NULL points
    pd.points = 256
    pd.params = 256
    pd.adam_m = 256
    pd.adam_v = 256
    pd.hp.alpha, pd.hp.w_iso, pd.hp.eta0, pd.hp.eta_growth = 5.56, 250.0, 5e-3, 1.1
    pd.hp.lambda0, pd.hp.lambda_growth, pd.hp.beta1, pd.hp.beta2 = 0.25, 1.5, 0.9, 0.999
    pd.hp.eps, pd.hp.e_max = 1e-8, 50
    pd.cg_tol = 1e-7
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.OK
    assert nb.value > 0
    pd.hp.beta1 = 1.0
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.EINVAL
    h = ctypes.c_void_p()
    pd.hp.beta1 = 0.9
    pd.workspace_bytes = 16
    pd.workspace = 256
    assert lib.pdg_problem_create(ctypes.byref(pd), None, ctypes.byref(h)) == L.ENOMEM
    # the keyframe lies in [0, frames)
    pd.keyframe = 3
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.EINVAL
    assert "keyframe" in L.last_error()
    pd.keyframe = 1
    nb1 = ctypes.c_size_t()
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb1)) == L.OK
    assert nb1.value > 0
    pd.keyframe = 0
    # X_0 optimisation needs both moments and a positive learning rate
    pd.template_adam_m = 256
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.EINVAL
    assert "X_0" in L.last_error()
    pd.template_adam_m = None
    # pruned grids need the conjugate-gradient preconditioner
    pd.prune_mask = 256
    pd.precond_method = L.PRECOND_METHODS["dct"]
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.EUNSUPPORTED
    assert "pruned" in L.last_error()
    pd.precond_method = L.PRECOND_METHODS["cg"]
    assert lib.pdg_problem_workspace(ctypes.byref(pd), ctypes.byref(nb)) == L.OK


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", L.LIB_PATH + ".absent")
    with pytest.raises(RuntimeError, match="no fallback"):
        L.lib()


def test_chamfer_noalloc_rejects_sizes_above_its_fixed_scratch():
    """The no-allocation Chamfer refuses, on the host and before touching any
    device, a pair whose workspace exceeds its fixed 64 MiB scratch."""
    lib = L.lib()
    nb = ctypes.c_size_t()
    assert lib.pdg_chamfer_workspace(600_000, 600_000, 1, ctypes.byref(nb)) == L.OK
    assert nb.value > 64 << 20
    st = lib.pdg_chamfer_noalloc(None, 600_000, None, 600_000, 5.56, 1, None, None, None, None,
                                 None, None)
    assert st == L.ENOMEM and "fixed scratch" in L.last_error()
    assert lib.pdg_chamfer_noalloc(None, 0, None, 10, 5.56, 0, None, None, None, None, None,
                                   None) == L.EINVAL
