"""ctypes binding of libpdg.so (include/pdg.h): argument marshalling only.

Every function takes and returns torch tensors on the current HIP device and
enqueues on torch's current stream; all arithmetic runs in the library's HIP
kernels.  If the library has not been built, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdg.so")
MAX_LEVELS = 16                # PDG_MAX_LEVELS of include/pdg.h

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, 1, 2, 3, 4
CHAMFER_MODES = {"fp32": 0, "bf16": 1, "bf16_screen": 1, "fp32cull": 2}
PRECOND_METHODS = {"cg": 0, "dct": 1}
STAGES = ("warp", "nn", "loss", "grad", "scatter", "precond", "adam")
# stage ids of pdg_step_stage: the seven stages and "precond_adam" (the last
# two as pdg_step runs them)
STAGE_IDS = {**{n: i for i, n in enumerate(STAGES)}, "precond_adam": 7, "template": 8}
BUFFERS = {"phat": 0, "xhat": 1, "nn": 2, "losses": 3, "wconf": 4, "grad": 5, "pgrad": 6,
           "gphat": 7, "gxhat": 8, "terms": 9, "lam": 10, "screen_tiles": 11, "nn0": 12,
           "loss0": 13, "gx0": 14, "pgx0": 15}


class PdgError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what} failed with status {status}: {msg}")
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("res", ctypes.c_int32 * MAX_LEVELS),
                ("channels", ctypes.c_int32), ("level_scale", ctypes.c_float)]


class Hyper(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("w_iso", ctypes.c_float), ("eta0", ctypes.c_float),
                ("eta_growth", ctypes.c_float), ("lambda0", ctypes.c_float),
                ("lambda_growth", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("e_max", ctypes.c_int32),
                ("mesh_lambda", ctypes.c_float), ("mesh_lr", ctypes.c_float)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_int32), ("n", ctypes.c_int64), ("points", ctypes.c_void_p),
                ("verts", ctypes.c_int32), ("template_verts", ctypes.c_void_p),
                ("n_edges", ctypes.c_int32), ("edges", ctypes.c_void_p),
                ("grid", GridDesc), ("hp", Hyper), ("chamfer_mode", ctypes.c_int32),
                ("precond_method", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("cg_tol", ctypes.c_double), ("prune_mask", ctypes.c_void_p),
                ("params", ctypes.c_void_p),
                ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("template_adam_m", ctypes.c_void_p), ("template_adam_v", ctypes.c_void_p),
                ("keyframe", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_F = ctypes.c_float
_D = ctypes.c_double
_SIGS = {
    "pdg_last_error": (ctypes.c_char_p, []),
    "pdg_version": (_I32, []),
    "pdg_grid_size": (_I64, [ctypes.POINTER(GridDesc)]),
    "pdg_deform": (_I32, [ctypes.POINTER(GridDesc), _P, _P, _I64, _P, _P]),
    "pdg_deform_backward_workspace": (_I32, [ctypes.POINTER(GridDesc), _I64, ctypes.POINTER(_SZ)]),
    "pdg_deform_backward": (_I32, [ctypes.POINTER(GridDesc), _P, _P, _I64, _P, _P, _P, _P, _SZ, _P]),
    "pdg_mesh_precondition_workspace": (_I32, [_I64, _I64, ctypes.POINTER(_SZ)]),
    "pdg_mesh_precondition": (_I32, [_I64, _P, _I64, _F, _I32, _I32, _D, _P, _P, _P, _SZ, _P]),
    "pdg_mesh_plan_create": (_I32, [_I64, _P, _I64, _F, _I32, _I32, _D, _P, _SZ, _P,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "pdg_mesh_plan_apply": (_I32, [ctypes.c_void_p, _P, _P, _P]),
    "pdg_mesh_plan_info": (_I32, [ctypes.c_void_p, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "pdg_mesh_plan_destroy": (_I32, [ctypes.c_void_p]),
    "pdg_mesh_partition": (_I32, [_I64, _P, _I64, _P, _P, _P, _P, _P]),
    "pdg_keyframe_workspace": (_I32, [_I32, ctypes.POINTER(_SZ)]),
    "pdg_keyframe": (_I32, [_P, _I32, _I64, _D, _P, _P, _P, _SZ, _P]),
    "pdg_chamfer_workspace": (_I32, [_I64, _I64, _I32, ctypes.POINTER(_SZ)]),
    "pdg_chamfer": (_I32, [_P, _I64, _P, _I64, _D, _I32, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "pdg_chamfer_noalloc": (_I32, [_P, _I64, _P, _I64, _D, _I32, _P, _P, _P, _P, _P, _P]),
    "pdg_chamfer_backward": (_I32, [_P, _I64, _P, _I64, _D, _P, _P, _P, _P, _P, _SZ, _P]),
    "pdg_precondition_workspace": (_I32, [ctypes.POINTER(GridDesc), _I32, _I32, ctypes.POINTER(_SZ)]),
    "pdg_precondition": (_I32, [ctypes.POINTER(GridDesc), ctypes.POINTER(_F), _P, _I32, _I32, _I32,
                                _D, _P, _SZ, _P]),
    "pdg_prune_mask_words": (_I32, [ctypes.POINTER(GridDesc), ctypes.POINTER(_I64)]),
    "pdg_prune_workspace": (_I32, [ctypes.POINTER(GridDesc), _I32, ctypes.POINTER(_SZ)]),
    "pdg_prune_mask": (_I32, [ctypes.POINTER(GridDesc), _I32, _I32, _P, _I64, _I32, _P, _P, _P, _SZ,
                              _P]),
    "pdg_precondition_pruned": (_I32, [ctypes.POINTER(GridDesc), ctypes.POINTER(_F), _P, _I32, _I32,
                                       _D, _P, _P, _SZ, _P]),
    "pdg_adam": (_I32, [ctypes.POINTER(GridDesc), _I32, ctypes.POINTER(_F), _F, _F, _F, _I32, _P,
                        _P, _P, _P, _P]),
    "pdg_problem_workspace": (_I32, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(_SZ)]),
    "pdg_problem_create": (_I32, [ctypes.POINTER(ProblemDesc), _P, ctypes.POINTER(_P)]),
    "pdg_step": (_I32, [_P, _I32, _P, _I32, _P]),
    "pdg_step_stage": (_I32, [_P, _I32, _P]),
    "pdg_batch_workspace": (_I32, [ctypes.POINTER(_P), _I32, ctypes.POINTER(_SZ)]),
    "pdg_batch_create": (_I32, [ctypes.POINTER(_P), _I32, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "pdg_batch_step": (_I32, [_P, ctypes.POINTER(_I32), _I32, _P]),
    "pdg_batch_destroy": (_I32, [_P]),
    "pdg_problem_destroy": (_I32, [_P]),
    "pdg_problem_buffer": (_I32, [_P, _I32, ctypes.POINTER(_P), ctypes.POINTER(_SZ)]),
    "pdg_problem_branch": (_I32, [_P, _I32, ctypes.POINTER(_P)]),
}
EXPORTS = tuple(_SIGS)


def lib():
    """Load libpdg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2509_18097_amd._build` (there is no fallback)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def last_error() -> str:
    return lib().pdg_last_error().decode()


def check(status: int, what: str):
    if status != OK:
        raise PdgError(status, what, last_error())


def grid_desc(res, level_scale=None, channels=3) -> GridDesc:
    res = tuple(int(r) for r in res)
    if not 1 <= len(res) <= MAX_LEVELS:
        raise ValueError(f"need 1..{MAX_LEVELS} levels, got {len(res)}")
    d = GridDesc()
    d.levels = len(res)
    for i, r in enumerate(res):
        d.res[i] = r
    d.channels = channels
    d.level_scale = 1.0 / len(res) if level_scale is None else float(level_scale)
    return d


def grid_size(res, channels=3) -> int:
    """Floats of one packed stack: channels (3: translation, 6: [z; t]) per cell."""
    return channels * sum(int(r) ** 3 for r in res)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def deform(grids: torch.Tensor, x: torch.Tensor, res, level_scale=None, out=None,
           channels=3) -> torch.Tensor:
    """x + level_scale * sum_l trilerp(G_l, x) (Eq. 1) for channels = 3; for
    channels = 6 (cells [z; t], Eq. 4-7) R(z^) x + t^.  x SoA (3, n) float32."""
    d = grid_desc(res, level_scale, channels)
    _dev(grids, torch.float32, "grids")
    _dev(x, torch.float32, "x")
    if grids.numel() != grid_size(res, channels) or x.dim() != 2 or x.shape[0] != 3:
        raise ValueError("grids must hold one packed stack and x must be (3, n)")
    out = torch.empty_like(x) if out is None else _dev(out, torch.float32, "out")
    check(lib().pdg_deform(ctypes.byref(d), _ptr(grids), _ptr(x), x.shape[1], _ptr(out), _stream()),
          "pdg_deform")
    return out


def deform_backward(grids, x, gout, res, level_scale=None, need_grids=True, need_x=True,
                    channels=3):
    """(dL/dG, dL/dx) for an upstream dL/dout (the adjoint of ``deform``)."""
    d = grid_desc(res, level_scale, channels)
    _dev(grids, torch.float32, "grids")
    _dev(x, torch.float32, "x")
    _dev(gout, torch.float32, "gout")
    n = x.shape[1]
    gg = torch.empty_like(grids) if need_grids else None
    gx = torch.empty_like(x) if need_x else None
    nb = ctypes.c_size_t()
    check(lib().pdg_deform_backward_workspace(ctypes.byref(d), n, ctypes.byref(nb)),
          "pdg_deform_backward_workspace")
    ws = _ws(nb.value, x.device) if need_grids else None
    check(lib().pdg_deform_backward(ctypes.byref(d), _ptr(grids), _ptr(x), n, _ptr(gout), _ptr(gg),
                                    _ptr(gx), _ptr(ws), nb.value if ws is not None else 0,
                                    _stream()), "pdg_deform_backward")
    return gg, gx


def mesh_precondition(g: torch.Tensor, edges: torch.Tensor, max_degree: int, lam: float = 16.0,
                      terms: int = 0, tol: float = 1e-8, out=None) -> torch.Tensor:
    """(I + lam L)^-2 g for the mesh Laplacian of edges (2, E) int32; g (3, V)
    float32; max_degree bounds every vertex degree (Sec. 3.2, 3.6).  One call
    builds a plan (synchronous) and applies it; see MeshPlan to apply many."""
    _dev(g, torch.float32, "g")
    _dev(edges, torch.int32, "edges")
    if g.dim() != 2 or g.shape[0] != 3 or edges.dim() != 2 or edges.shape[0] != 2:
        raise ValueError("g must be (3, V) and edges (2, E)")
    v, e = g.shape[1], edges.shape[1]
    out = torch.empty_like(g) if out is None else _dev(out, torch.float32, "out")
    nb = ctypes.c_size_t()
    check(lib().pdg_mesh_precondition_workspace(v, e, ctypes.byref(nb)),
          "pdg_mesh_precondition_workspace")
    ws = _ws(nb.value, g.device)
    check(lib().pdg_mesh_precondition(v, _ptr(edges) if e > 0 else None, e, float(lam),
                                      int(max_degree), int(terms), float(tol), _ptr(g), _ptr(out),
                                      _ptr(ws), nb.value, _stream()), "pdg_mesh_precondition")
    return out


def mesh_partition(edges, vertices: int):
    """The vertex parts a mesh plan of edges ((2, E) host int array) would use
    (host only): (part_off, part_core, local_vertex, local_dist, k, local_max),
    the arrays None when the plan runs one term per launch."""
    import numpy as np
    e = np.ascontiguousarray(edges, dtype=np.int32)
    if e.ndim != 2 or e.shape[0] != 2:
        raise ValueError("edges must be (2, E)")
    ne = e.shape[1]
    ep = e.ctypes.data if ne > 0 else None
    sizes = np.zeros(4, dtype=np.int64)
    check(lib().pdg_mesh_partition(int(vertices), ep, ne, None, None, None, None,
                                   sizes.ctypes.data), "pdg_mesh_partition")
    np_, nl, k, lmax = (int(x) for x in sizes)
    if np_ == 0:
        return None, None, None, None, k, lmax
    po = np.zeros(np_ + 1, np.int32)
    pc = np.zeros(np_, np.int32)
    lv = np.zeros(nl, np.int32)
    ld = np.zeros(nl, np.int32)
    check(lib().pdg_mesh_partition(int(vertices), ep, ne, po.ctypes.data, pc.ctypes.data,
                                   lv.ctypes.data, ld.ctypes.data, sizes.ctypes.data),
          "pdg_mesh_partition")
    return po, pc, lv, ld, k, lmax


class MeshPlan:
    """A built mesh preconditioner (pdg_mesh_plan_*): the series coefficients
    and the vertex parts of one edge list, in a device workspace it keeps."""

    def __init__(self, edges: torch.Tensor, vertices: int, max_degree: int, lam: float = 16.0,
                 terms: int = 0, tol: float = 1e-8):
        _dev(edges, torch.int32, "edges")
        if edges.dim() != 2 or edges.shape[0] != 2:
            raise ValueError("edges must be (2, E)")
        self.V, e = int(vertices), edges.shape[1]
        nb = ctypes.c_size_t()
        check(lib().pdg_mesh_precondition_workspace(self.V, e, ctypes.byref(nb)),
              "pdg_mesh_precondition_workspace")
        self._ws = _ws(nb.value, edges.device)
        h = ctypes.c_void_p()
        check(lib().pdg_mesh_plan_create(self.V, _ptr(edges) if e > 0 else None, e, float(lam),
                                         int(max_degree), int(terms), float(tol), _ptr(self._ws),
                                         nb.value, _stream(), ctypes.byref(h)),
              "pdg_mesh_plan_create")
        self._h = h
        t, p = _I32(), _I32()
        check(lib().pdg_mesh_plan_info(self._h, ctypes.byref(t), ctypes.byref(p)),
              "pdg_mesh_plan_info")
        self.terms, self.parts = t.value, p.value

    def apply(self, g: torch.Tensor, out=None) -> torch.Tensor:
        _dev(g, torch.float32, "g")
        if g.dim() != 2 or g.shape != (3, self.V):
            raise ValueError(f"g must be (3, {self.V})")
        out = torch.empty_like(g) if out is None else _dev(out, torch.float32, "out")
        check(lib().pdg_mesh_plan_apply(self._h, _ptr(g), _ptr(out), _stream()),
              "pdg_mesh_plan_apply")
        return out

    def close(self):
        if self._h:
            lib().pdg_mesh_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def keyframe(points: torch.Tensor, gamma: float = 0.001):
    """Keyframe selection (Sec. 3.5, Eq. 19-20) of points (F, 3, N) float32:
    returns (t_key int32 (1,), occupied-voxel counts int64 (F,)) on the device."""
    _dev(points, torch.float32, "points")
    if points.dim() != 3 or points.shape[1] != 3:
        raise ValueError("points must be (F, 3, N)")
    f, n = points.shape[0], points.shape[2]
    nb = ctypes.c_size_t()
    check(lib().pdg_keyframe_workspace(f, ctypes.byref(nb)), "pdg_keyframe_workspace")
    ws = _ws(nb.value, points.device)
    key = torch.empty(1, dtype=torch.int32, device=points.device)
    counts = torch.empty(f, dtype=torch.int64, device=points.device)
    check(lib().pdg_keyframe(_ptr(points), f, n, float(gamma), _ptr(counts), _ptr(key), _ptr(ws),
                             nb.value, _stream()), "pdg_keyframe")
    return key, counts


def chamfer(a, b, alpha=5.56, mode="fp32", dir_weight=None, need_grad=False):
    """Robust Chamfer (Eq. 11-13).  Returns (loss float64 (2,), nn_a, nn_b, ga or None)."""
    _dev(a, torch.float32, "a")
    _dev(b, torch.float32, "b")
    n, m = a.shape[1], b.shape[1]
    md = CHAMFER_MODES[mode]
    nb = ctypes.c_size_t()
    check(lib().pdg_chamfer_workspace(n, m, md, ctypes.byref(nb)), "pdg_chamfer_workspace")
    ws = _ws(nb.value, a.device)
    loss = torch.empty(2, dtype=torch.float64, device=a.device)
    nn_a = torch.empty(n, dtype=torch.int32, device=a.device)
    nn_b = torch.empty(m, dtype=torch.int32, device=a.device)
    ga = torch.empty_like(a) if need_grad else None
    if dir_weight is not None:
        dir_weight = _dev(dir_weight, torch.float64, "dir_weight")
    check(lib().pdg_chamfer(_ptr(a), n, _ptr(b), m, float(alpha), md, _ptr(dir_weight), _ptr(loss),
                            _ptr(nn_a), _ptr(nn_b), _ptr(ga), _ptr(ws), nb.value, _stream()),
          "pdg_chamfer")
    return loss, nn_a, nn_b, ga


def chamfer_noalloc(a, b, alpha=5.56, mode="fp32", dir_weight=None, need_grad=False,
                    out=None):
    """pdg_chamfer on the library's fixed device scratch (no workspace
    allocated).  ``out`` = (loss, nn_a, nn_b, ga) reuses caller tensors so that
    nothing is allocated here either.  Returns (loss, nn_a, nn_b, ga or None)."""
    _dev(a, torch.float32, "a")
    _dev(b, torch.float32, "b")
    n, m = a.shape[1], b.shape[1]
    if out is None:
        out = (torch.empty(2, dtype=torch.float64, device=a.device),
               torch.empty(n, dtype=torch.int32, device=a.device),
               torch.empty(m, dtype=torch.int32, device=a.device),
               torch.empty_like(a) if need_grad else None)
    loss, nn_a, nn_b, ga = out
    if dir_weight is not None:
        dir_weight = _dev(dir_weight, torch.float64, "dir_weight")
    check(lib().pdg_chamfer_noalloc(_ptr(a), n, _ptr(b), m, float(alpha), CHAMFER_MODES[mode],
                                    _ptr(dir_weight), _ptr(loss), _ptr(nn_a), _ptr(nn_b), _ptr(ga),
                                    _stream()), "pdg_chamfer_noalloc")
    return loss, nn_a, nn_b, ga


def chamfer_backward(a, b, nn_a, nn_b, dir_weight, alpha=5.56):
    """d/da of dir_weight[0]*loss[0] + dir_weight[1]*loss[1] from saved indices."""
    _dev(a, torch.float32, "a")
    _dev(b, torch.float32, "b")
    _dev(nn_a, torch.int32, "nn_a")
    _dev(nn_b, torch.int32, "nn_b")
    _dev(dir_weight, torch.float64, "dir_weight")
    n, m = a.shape[1], b.shape[1]
    nb = ctypes.c_size_t()
    check(lib().pdg_chamfer_workspace(n, m, 0, ctypes.byref(nb)), "pdg_chamfer_workspace")
    ws = _ws(nb.value, a.device)
    ga = torch.empty_like(a)
    check(lib().pdg_chamfer_backward(_ptr(a), n, _ptr(b), m, float(alpha), _ptr(nn_a), _ptr(nn_b),
                                     _ptr(dir_weight), _ptr(ga), _ptr(ws), nb.value, _stream()),
          "pdg_chamfer_backward")
    return ga


def precondition(g, res, lambdas, batch=1, method="cg", iters=0, tol=1e-7, channels=3):
    """In place g <- (I + lambda_l L_l)^-2 g per level and channel (Eq. 3)."""
    d = grid_desc(res, 1.0, channels)
    _dev(g, torch.float32, "g")
    if g.numel() != batch * grid_size(res, channels):
        raise ValueError("g must hold `batch` packed stacks")
    md = PRECOND_METHODS[method]
    lam = (ctypes.c_float * MAX_LEVELS)(*[float(v) for v in lambdas])
    nb = ctypes.c_size_t()
    check(lib().pdg_precondition_workspace(ctypes.byref(d), batch, md, ctypes.byref(nb)),
          "pdg_precondition_workspace")
    ws = _ws(nb.value, g.device)
    check(lib().pdg_precondition(ctypes.byref(d), lam, _ptr(g), batch, md, iters, tol, _ptr(ws),
                                 nb.value, _stream()), "pdg_precondition")
    return g


def prune_mask_words(res) -> int:
    """uint32 words of one stack's pruning mask (one bit per cell and level)."""
    d = grid_desc(res, 1.0)
    w = ctypes.c_int64()
    check(lib().pdg_prune_mask_words(ctypes.byref(d), ctypes.byref(w)), "pdg_prune_mask_words")
    return w.value


def prune_mask(points: torch.Tensor, res, span: int = 2, halo: int = 3):
    """Pruned grids (Sec. 3.6): kept-cell masks of the stacks b = 0 .. F - span,
    stack b pruned by frames b .. b + span - 1 of points (F, 3, N) float32.
    Returns (mask int32 (stacks, words) holding the uint32 bits, kept cells
    int64 (stacks, levels))."""
    _dev(points, torch.float32, "points")
    if points.dim() != 3 or points.shape[1] != 3:
        raise ValueError("points must be (F, 3, N)")
    stacks = points.shape[0] - span + 1
    if stacks < 0:
        raise ValueError("fewer frames than span - 1")
    d = grid_desc(res, 1.0)
    words = prune_mask_words(res)
    mask = torch.empty((max(stacks, 0), words), dtype=torch.int32, device=points.device)
    active = torch.empty((max(stacks, 0), len(res)), dtype=torch.int64, device=points.device)
    nb = ctypes.c_size_t()
    check(lib().pdg_prune_workspace(ctypes.byref(d), max(stacks, 0), ctypes.byref(nb)),
          "pdg_prune_workspace")
    ws = _ws(nb.value, points.device)
    check(lib().pdg_prune_mask(ctypes.byref(d), max(stacks, 0), span, _ptr(points), points.shape[2],
                               halo, _ptr(mask), _ptr(active), _ptr(ws), nb.value, _stream()),
          "pdg_prune_mask")
    return mask, active


def precondition_pruned(g, res, lambdas, mask, batch=1, iters=0, tol=1e-7):
    """In place g <- (I + lambda_l L_S)^-2 g on the kept cells of every level
    (Eq. 3 on pruned grids), 0 on pruned cells; mask as ``prune_mask``."""
    d = grid_desc(res, 1.0)
    _dev(g, torch.float32, "g")
    _dev(mask, torch.int32, "mask")
    if g.numel() != batch * grid_size(res):
        raise ValueError("g must hold `batch` packed stacks")
    if mask.numel() != batch * prune_mask_words(res):
        raise ValueError("mask must hold `batch` stacks of prune_mask_words(res) words")
    lam = (ctypes.c_float * MAX_LEVELS)(*[float(v) for v in lambdas])
    nb = ctypes.c_size_t()
    check(lib().pdg_precondition_workspace(ctypes.byref(d), batch, PRECOND_METHODS["cg"],
                                           ctypes.byref(nb)), "pdg_precondition_workspace")
    ws = _ws(nb.value, g.device)
    check(lib().pdg_precondition_pruned(ctypes.byref(d), lam, _ptr(g), batch, iters, tol,
                                        _ptr(mask), _ptr(ws), nb.value, _stream()),
          "pdg_precondition_pruned")
    return g


def adam(theta, m, v, g, res, lrs, step, batch=1, beta1=0.9, beta2=0.999, eps=1e-8, channels=3):
    d = grid_desc(res, 1.0, channels)
    for t, nm in ((theta, "theta"), (m, "m"), (v, "v"), (g, "g")):
        _dev(t, torch.float32, nm)
    lr = (ctypes.c_float * MAX_LEVELS)(*[float(x) for x in lrs])
    check(lib().pdg_adam(ctypes.byref(d), batch, lr, beta1, beta2, eps, step, _ptr(theta), _ptr(m),
                         _ptr(v), _ptr(g), _stream()), "pdg_adam")
