"""CPU oracle for the matrix-completion primal-dual interior-point method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the GPU library and its
Python binding) imports, calls, links or executes this package; only the
tests, the smoke check and the benchmark's CPU-baseline leg do.

Everything here is plain, slow and written to be checked by eye against
the paper (Yamashita & Nakata, "Fast implementation for semidefinite
programs with positive matrix completion"):

  symbolic    chordal extension of the aggregate sparsity pattern for a
              given elimination order, elimination tree, supernodes used as
              the clique sequence C_1..C_l with S_r / U_r (Sections 2.1, 3.1)
  completion  max-determinant completion through the two-clique formula of
              the validity proof (Section 3.1), Algorithm 1 (Cholesky factor
              of the inverse of the completion), the textbook route
              chol(inv(X^)) for comparison, and the earlier sparse
              factorisation X^ = L^T D L (Section 2.1)
  scm         the Schur complement matrix from its definition (eq. SCM) and
              the right-hand side of the Schur complement equation
  pdipm       a dense HKM primal-dual interior-point method (Section 2.2,
              Steps 0-4) and the matrix-completion variant that keeps X only
              on the extended pattern (eqs. newdX2, primal_length2)
  checks      brute-force max-cut and closed-form SDP values

All floating point is IEEE float64.  Readings of garbled or silent passages
of the paper are listed in the module docstrings where they are used.
"""
from .symbolic import Chordal, chordal_structure, sym_sparse, aggregate_pattern  # noqa: F401
from .completion import (maxdet_complete, algorithm1, lhat_textbook,  # noqa: F401
                         completion_by_vertex, sparse_factors)
from .scm import dense_scm, scm_rhs, scm_kron  # noqa: F401
from .pdipm import (Params, dense_pdipm, mc_pdipm, mc_direction, dense_state_metrics,  # noqa: F401
                    step_length_dense, step_length_cliques)
from .checks import brute_force_maxcut, cycle_sdp_value  # noqa: F401
