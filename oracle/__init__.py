"""CPU oracle for the regularized normal equations (FP64, numpy/scipy).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or executes it, and
the two share no code: the oracle builds explicit sparse matrices straight
from the paper's definitions and solves with plain library primitives.

What it computes, for each outer weighting D and regularization parameter
lambda (paper, Section 1 eq. (LSreg) and Section 3.2 eq. (normal)):

    x*(lambda) = argmin ||A x - b||^2 + lambda^2 ||D L x||^2
               = (A^T A + lambda^2 L^T D^2 L)^{-1} A^T b

together with the L-curve pair (||A x* - b||, ||D L x*||) (Section 1), and,
as an independent reference for the preconditioned solver, the multigrid
V-cycle of Algorithm 1 built on the one-sided hierarchies A_k = A_{k-1} P,
M_k = M_{k-1} P of Section 3.2, with a Jacobi-preconditioned Chebyshev
smoother and an exact coarsest solve.

Modules:
  operators  -- explicit A (blur, any boundary), L, D, K(lambda)
  direct     -- dense, stacked least-squares, FFT and DCT closed-form solves
  multigrid  -- interpolation, one-sided hierarchy, smoother, V-cycle
  pcg        -- preconditioned conjugate gradients and reference solves

Every function is pinned by a `-m "not gpu"` test against a value fixed
independently of this package (closed forms, textbook stencils, brute force,
library routines, invariants).
"""
