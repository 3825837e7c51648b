"""FP64 CPU oracle for the structured-operator conic solver.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, links or calls
this package; only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library: the only common
module is ``workloads`` (seeded input draws, no solver arithmetic).

What it computes (plain, slow, obviously correct, float64 throughout):

* ``program``  -- the cone programs of the paper's examples written out
  explicitly in the sign convention ``minimize c^T x  s.t.  A x + s = b, s in K``
  (eq. (1) with ``A -> -A``), with ``K`` a product of a nonnegative orthant and
  second-order cones, and the matrix ``I + A^T A`` factored directly (dense
  Cholesky, or banded Cholesky for a convolution block).
* ``cones``    -- closed-form Euclidean projections onto those cones.
* ``equil``    -- the diagonal equilibration the iteration runs on (a reading:
  the paper leaves preconditioning open).
* ``scs``      -- the homogeneous self-dual embedding ADMM iteration the paper
  runs ("SCS", Sections II-D and V-B), with the linear-subspace step solved
  exactly through the factorisation instead of by conjugate gradients.
* ``regls``    -- the closed-form solution of regularized least squares
  (Section V-A), computed by a direct factorisation.
* ``polish``   -- a textbook active-set step that turns the iterative result into
  an exact optimum with a KKT certificate (nonnegative least squares / lasso).

Every function cites the passage of the paper it follows; where the paper is
silent the reading taken is stated in the function's docstring.
"""
from .cones import proj_nonneg, proj_soc, proj_cone, in_cone
from .program import ConeProgram, deconv_program, lasso_program, dense_program, conv_lasso_program
from .equil import Scaling, equilibrate, scaled_program
from .scs import scs_solve, ScsResult, hsde_subspace_step, prepare
from .polish import polish_deconv, polish_lasso, deconv_objective, lasso_objective
from .regls import regls_solution, regls_rhs, regls_apply_normal, regls_objective

__all__ = [
    "proj_nonneg", "proj_soc", "proj_cone", "in_cone",
    "ConeProgram", "deconv_program", "lasso_program", "dense_program", "conv_lasso_program",
    "regls_solution", "regls_rhs", "regls_apply_normal", "regls_objective",
    "Scaling", "equilibrate", "scaled_program",
    "scs_solve", "ScsResult", "hsde_subspace_step", "prepare",
    "polish_deconv", "polish_lasso", "deconv_objective", "lasso_objective",
]
