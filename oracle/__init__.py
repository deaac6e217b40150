"""CPU oracle for the mortar-contact block-AMG solve.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 restatement of
the method for checking the GPU library; only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import it.  It shares no code with
the GPU library (it never imports it and the library never imports this).

Modules:
  hierarchy  -- Dirichlet detection, node graph, aggregation, the multiplier
                aggregation of Alg. 1, tentative transfers, Galerkin blocks,
                smoother data, coarsest-level inverse.
  smoother   -- CheapSIMPLE sweep (Alg. 3 with Jacobi / diagonal Schur
                inverses) and its adjoint.
  vcycle     -- recursive V-cycle (Fig. 2a) and its transpose.
  fgmres     -- right-preconditioned flexible GMRES(m) with CGS2.
  adjoint    -- adjoint solve and gradients w.r.t. b and the nonzeros of K.

Where the paper is silent the oracle follows one documented reading; each
function names the passage it follows.
"""
from .hierarchy import AMGOptions, Level, build_hierarchy
from .vcycle import vcycle
from .fgmres import fgmres
from .adjoint import solve_with_adjoint, grad_K_values

__all__ = ["AMGOptions", "Level", "build_hierarchy", "vcycle", "fgmres", "solve_with_adjoint", "grad_K_values"]
