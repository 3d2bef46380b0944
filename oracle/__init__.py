"""Plain FP64 CPU oracle for the dual-smoothing method (P-APG) on least-squares convex regression.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute anything in
this package: only the tests, the smoke check of the package entry file and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library (no kernels, headers, helpers,
constants or pre/post-processing); both consume the same seeded inputs from the workload
generators, which contain none of the method's arithmetic.

Contents
--------
``papg``   the method itself: the matrix-free constraint operator C and its adjoint, the closed-form
           Step 1 for the singleton partition (K = N), the Lipschitz constant by power iteration,
           the P-APG loop, the stopping report and the feasible-repair certificate.
``exact``  independent exact solvers for tiny N that build A1 and A2 explicitly from the
           T_l blocks of Definition ``def:A1A2``: the regularized dual as a non-negative least
           squares problem (Lawson-Hanson, via scipy) and the unregularized estimator of
           eq. ``original`` as a QP (SLSQP, via scipy).
``continuation``  the outer loop of Section 2.4.1 (gamma_t, delta_t -> 0 with warm starts).
``blocks`` P-APG with K-block partial dualization (Section 2.1): only the pairs between blocks are
           dualized, and Step 1 solves each block's QP exactly (NNLS on the block's dual).

All arithmetic is float64 with numpy's default round-to-nearest.  Each function cites the
passage of the paper (Aybat & Wang, "A Parallelizable Dual Smoothing Method for Large Scale
Convex Regression Problems", arXiv:1608.02227) that it follows.
"""
from .papg import (  # noqa: F401
    pair_residual,
    pair_adjoint,
    primal_from_dual,
    dual_objective,
    primal_objective,
    lipschitz,
    fista_schedule,
    papg,
    kkt_report,
    repair_certificate,
)
from .exact import explicit_constraints, exact_solve, exact_ls  # noqa: F401
from .continuation import continuation  # noqa: F401
