"""CPU oracle for the deform-and-match step of Preconditioned Deformation Grids.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of what the method computes, in float64 numpy, used to check the
HIP path.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never does, and this package imports
nothing from the product package.

Modules (each function cites the passage of the paper it follows):

* ``warp``      -- multi-resolution trilinear deformation (Sec. 3.1, Eq. 1),
                   its grid adjoint and position Jacobian.
* ``cayley``    -- six-channel cells [z; t] with the Cayley rotation (Sec. 3.3,
                   Eq. 4-7): warp x' = R(z^) x + t^ and both adjoints.
* ``chamfer``   -- robust Chamfer distance (Sec. 3.4, Eq. 11-13): brute-force
                   nearest neighbours, per-direction losses and gradients.
* ``precond``   -- grid Sobolev preconditioner (I + lambda L)^-2 (Sec. 3.2,
                   Eq. 3): dense Cholesky and the DCT-II closed form.
* ``prune``     -- pruned grids (Sec. 3.6): active cells by occupancy and a
                   three-cell halo, the preconditioner on the induced graph.
* ``adam``      -- Adam with bias correction (Sec. 3.6).
* ``keyframe``  -- keyframe selection by weighted 128^3 occupancy (Sec. 3.5,
                   Eq. 19-20).
* ``mesh``      -- the mesh-vertex preconditioner (I + lambda L)^-2 with the
                   mesh Laplacian (Sec. 3.2, 3.6).
* ``sequence``  -- isometry loss (Eq. 18), confidence weights (Eq. 15-17),
                   loss assembly (Eq. 9, 14) and one full optimisation step.

Readings of the paper where it is silent or ambiguous are listed in the
module docstrings where they are used.
"""
from . import warp, cayley, chamfer, precond, adam, sequence, keyframe, mesh, prune  # noqa: F401
