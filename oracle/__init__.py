"""FP64 CPU oracle for the multiscale spectral multigrid solve path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or executes it, and
this package imports nothing from the product path.

Each module follows the paper (arXiv 2403.19342) step by step, in float64,
with plain NumPy/SciPy building blocks and no blocking or fusion:

  assembly   Section 2.2: harmonic-mean transmissibilities, the TPFA matrix A
             obtained by velocity elimination, the weight S = diag(tr K~).
  spectral   Section 3: local generalized eigenproblems (eq. spepb) on the
             coarse elements, their restriction to the coarse space for the
             coarser levels (eq. spectral cc), the Galerkin chain.
  smoothers  Section 5: block-Jacobi smoothers with incomplete Cholesky blocks.
  vcycle     Algorithm 1 (three-grid iteration) applied recursively, with the
             pseudo-inverse at the coarsest level.
  pcg        Preconditioned conjugate gradients around the V-cycle.
  gmres      Restarted flexible GMRES around the V-cycle (the outer solver
             of the paper's experiments, Section 5).
  flux       Section 2.2: velocity recovery v = M_t^{-1} B^T p (the
             two-point flux of eq. (velocity)) and the cell mass balance.
  impes      Section 6: the two-phase model (relative permeabilities,
             total mobility, fractional flow) and the improved IMPES step
             with upstream-weighted explicit saturation sub-steps.
  cnn        Extension, not in the paper: the 3D CNN that predicts start
             blocks for the level-2 eigenproblems, its subspace loss and
             gradients (forward and backward written out in float64).
  dense      Brute-force dense references for tiny grids.
"""
from .assembly import Grid, transmissibilities, assemble, weight_diag, neumann_local
from .spectral import Hierarchy, build_hierarchy, cluster_cut, threshold_target
from .vcycle import Preconditioner
from .pcg import pcg
from .gmres import fgmres
from .flux import recover_flux, mass_balance
from . import impes

__all__ = [
    "Grid", "transmissibilities", "assemble", "weight_diag", "neumann_local",
    "Hierarchy", "build_hierarchy", "cluster_cut", "threshold_target", "Preconditioner", "pcg", "fgmres",
    "recover_flux", "mass_balance", "impes",
]
