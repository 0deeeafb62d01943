"""Preconditioned conjugate gradients and reference solves (FP64).

pcg() is the textbook Hestenes-Stiefel recurrence with a symmetric positive
definite preconditioner.  Iterations are counted as the number of products
K p taken until the recursive residual meets the target; the target is
tol * ||A^T b|| (relative) or tol (absolute, as in the paper's Section 3.3).
"""
from __future__ import annotations

import numpy as np

from . import direct
from . import operators as ops
from .multigrid import Hierarchy, KrylovVCycle, SparseOp, VCycle


def pcg(K, f, M=None, x0=None, tol=1e-8, maxit=10000, absolute=False,
        stall=None, flexible=False):
    """Solve K x = f.  Returns (x, iterations, final recursive ||r||, history).

    stall: stop when the best residual has not decreased for this many steps
    (used to iterate to the floating-point floor).
    flexible: Polak-Ribiere beta = z_new . (r_new - r_old) / (r_old . z_old)
    (flexible CG, Notay 2000), for a preconditioner that is not the same
    linear map at every application (e.g. a V-cycle evaluated in reduced
    precision); with a fixed SPD M it gives the same iterates as the
    standard beta.
    """
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - K(x) if x0 is not None else f.copy()
    target = tol if absolute else tol * np.linalg.norm(f)
    hist = [np.linalg.norm(r)]
    if hist[0] <= target:
        return x, 0, hist[0], hist
    z = r.copy() if M is None else M(r)
    p = z.copy()
    gamma = float(r @ z)
    best, since = hist[0], 0
    for it in range(1, maxit + 1):
        q = K(p)
        alpha = gamma / float(p @ q)
        x += alpha * p
        r_old = r.copy() if flexible else None
        r -= alpha * q
        nr = float(np.linalg.norm(r))
        hist.append(nr)
        if nr <= target:
            return x, it, nr, hist
        if stall is not None:
            if nr < best:
                best, since = nr, 0
            else:
                since += 1
                if since >= stall:
                    return x, it, nr, hist
        z = r.copy() if M is None else M(r)
        gnew = float(r @ z)
        if flexible:
            beta = float(z @ (r - r_old)) / gamma
        else:
            beta = gnew / gamma
        p = z + beta * p
        gamma = gnew
    return x, maxit, hist[-1], hist


class DeblurOracle:
    """All oracle objects for one deblurring workload and outer weighting."""

    def __init__(self, nv, nh, taps_v, taps_h, bc, lbc, d, levels=1):
        self.nv, self.nh = nv, nh
        self.taps_v, self.taps_h = np.asarray(taps_v), np.asarray(taps_h)
        self.bc, self.lbc = bc, lbc
        self.d = np.asarray(d, dtype=np.float64)
        self.A = ops.KronBlur(ops.blur_matrix_1d(taps_v, nv, bc),
                              ops.blur_matrix_1d(taps_h, nh, bc))
        self.M = ops.regularizer(self.d, nv, nh, lbc)
        self.levels = levels
        self._H = None

    @property
    def H(self) -> Hierarchy:
        if self._H is None:
            self._H = Hierarchy(self.A, self.M, self.nv, self.nh, self.levels,
                                self.lbc == "periodic")
        return self._H

    def rhs(self, b):
        return self.A.rmatvec(b)

    def K(self, lam):
        M = self.M
        return lambda v: self.A.rmatvec(self.A.matvec(v)) + \
            lam * lam * (M.T @ (M @ v))

    def pair(self, x, b):
        return ops.lcurve_pair(self.A.matvec, self.M, x, b)

    def vcycle(self, lam, nu=2, ratio=4.0) -> VCycle:
        return VCycle(self.H, lam, nu, ratio)

    def unit_weights(self) -> bool:
        return bool(np.all(self.d == 1.0))

    def reference(self, b, lam, floor=1e-14, maxit=20000):
        """x*(lambda) to the FP64 floor.

        D = I with a matching boundary pair: DFT / DCT closed form.
        Otherwise: CG preconditioned by the exact D = I inverse, run until
        the relative residual reaches `floor` or stops decreasing.
        Returns (x, relative residual of the normal equations).
        """
        f = self.rhs(b)
        K = self.K(lam)
        pair = (self.bc, self.lbc)
        if self.unit_weights() and pair == ("periodic", "periodic"):
            x = direct.solve_fft(self.taps_v, self.taps_h, self.nv, self.nh,
                                 b, lam)
        elif self.unit_weights() and pair == ("reflective", "neumann"):
            x = direct.solve_dct(self.taps_v, self.taps_h, self.nv, self.nh,
                                 b, lam)
        elif pair in (("periodic", "periodic"), ("reflective", "neumann")):
            Minv = direct.spectral_inverse(self.taps_v, self.taps_h, self.nv,
                                           self.nh, self.bc, self.lbc, lam)
            x, _, _, _ = pcg(K, f, Minv, tol=floor, maxit=maxit, stall=60)
        else:
            x, _, _, _ = pcg(K, f, None, tol=floor, maxit=maxit, stall=200)
        rel = float(np.linalg.norm(f - K(x)) / np.linalg.norm(f))
        return x, rel

    def mg_pcg(self, b, lam, tol=1e-8, nu=2, ratio=4.0, x0=None,
               maxit=10000, absolute=False):
        """PCG preconditioned by the V-cycle: the reference for the
        preconditioned solver's iteration counts."""
        V = self.vcycle(lam, nu, ratio)
        return pcg(self.K(lam), self.rhs(b), V, x0=x0, tol=tol, maxit=maxit,
                   absolute=absolute)

    def krylov_mg_pcg(self, b, lam, tol=1e-8, nu_pre=2, nu_post=1, x0=None,
                      maxit=10000, absolute=False):
        """Flexible PCG preconditioned by the V(nu_pre, nu_post) cycle with
        diagonally preconditioned CG relaxation (the paper's preconditioner,
        Section 3.2; the paper runs it under FGMRES)."""
        V = KrylovVCycle(self.H, lam, nu_pre, nu_post)
        return pcg(self.K(lam), self.rhs(b), V, x0=x0, tol=tol, maxit=maxit,
                   absolute=absolute, flexible=True)


class CtOracle(DeblurOracle):
    """Oracle objects for one tomography workload and outer weighting: the
    same normal equations (paper Sec. 3.2) with a general sparse A (m x n,
    the projector handed over by the generator) and the same one-sided
    hierarchy A_{k+1} = A_k P (Sec. 3.2), formed here with SciPy products."""

    def __init__(self, A, N, lbc, d, levels=1):
        self.nv = self.nh = N
        self.taps_v = self.taps_h = None
        self.bc, self.lbc = "ct", lbc
        self.d = np.asarray(d, dtype=np.float64)
        self.A = SparseOp(A)
        self.M = ops.regularizer(self.d, N, N, lbc)
        self.levels = levels
        self._H = None

    def reference(self, b, lam, floor=1e-13, maxit=20000):
        """x*(lambda): a dense Cholesky solve of the normal equations for
        n <= 4096, otherwise CG preconditioned by this oracle's V-cycle run
        to `floor` or until it stops decreasing.
        Returns (x, relative residual of the normal equations)."""
        import scipy.linalg as sla
        f = self.rhs(b)
        K = self.K(lam)
        n = self.nv * self.nh
        if n <= 4096:
            A = self.A.explicit()
            Kd = (A.T @ A).toarray() + lam * lam * (self.M.T @ self.M).toarray()
            x = sla.cho_solve(sla.cho_factor(Kd), f)
        else:
            x, _, _, _ = pcg(K, f, self.vcycle(lam), tol=floor, maxit=maxit,
                             stall=60)
        rel = float(np.linalg.norm(f - K(x)) / np.linalg.norm(f))
        return x, rel


__all__ = ["pcg", "DeblurOracle", "CtOracle", "SparseOp"]
