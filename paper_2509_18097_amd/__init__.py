"""MI355X (gfx950) deform-and-match step of Preconditioned Deformation Grids.

The compute path lives in ``libpdg.so`` (hand-written HIP kernels behind the
C ABI of ``include/pdg.h``).  This package is the thin Python side: the
ctypes binding (``_lib``), the autograd functions (``autograd``), the
per-request problem object (``problem``) and the serving loop (``serve``).
Importing the package does not load the library; the first call does, and
raises if it has not been built (``python -m paper_2509_18097_amd._build``).
"""
from ._lib import PdgError, grid_size  # noqa: F401

__all__ = ["PdgError", "grid_size"]
