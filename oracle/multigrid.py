"""Multigrid V-cycle for K(lambda) = A^T A + lambda^2 M^T M (FP64).

Follows the paper's Section 3.2 construction: interpolation operators P_k
are built for the diffusion-like part L^T D^2 L, and the coarse operators
are never formed from A^T A.  Instead the one-sided hierarchies
A_1 = A, A_{k+1} = A_k P_k and M_1 = D L, M_{k+1} = M_k P_k are stored, and
the level-k operator is applied in two stages, x -> (A_k x, M_k x) -> back
through the transposes.  diag(A_k^T A_k) is the column sums of squares of
A_k and diag(M_k^T M_k) those of M_k.  One V-cycle is Algorithm 1 with
gamma = 1, R_k = P_k^T, and an exact solve on the coarsest level.

Interpolation here is geometric (vertex-centred linear in each direction,
P = P_h (x) P_v) rather than the paper's Ruge-Stueben choice, and the
relaxation is a Jacobi-preconditioned Chebyshev polynomial (the same
polynomial before and after the coarse correction, so that the cycle is a
symmetric positive definite preconditioner for plain CG) rather than the
paper's diagonally preconditioned CG, which would need a flexible Krylov
method.  The Chebyshev interval is [rho/alpha, rho], with rho the
Gershgorin bound max_i sum_j |K_ij| / K_ii of the Jacobi-scaled operator.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .operators import KronBlur


def interpolation_1d(n: int, periodic: bool) -> sp.csr_matrix:
    """Vertex-centred linear interpolation from n/2 coarse points to n.

    Coarse point I sits on fine point 2I (weight 1).  Odd fine point 2I+1
    averages its two coarse neighbours; the last odd point wraps to coarse
    point 0 when periodic and otherwise copies its single neighbour, so that
    P 1 = 1 in both cases.
    """
    if n % 2 or n < 4:
        raise ValueError("interpolation needs an even size >= 4")
    nc = n // 2
    rows, cols, vals = [], [], []
    for I in range(nc):
        rows.append(2 * I)
        cols.append(I)
        vals.append(1.0)
        f = 2 * I + 1
        if I + 1 < nc:
            rows += [f, f]
            cols += [I, I + 1]
            vals += [0.5, 0.5]
        elif periodic:
            rows += [f, f]
            cols += [I, 0]
            vals += [0.5, 0.5]
        else:
            rows.append(f)
            cols.append(I)
            vals.append(1.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


class SparseOp:
    """A general sparse forward operator with the same interface as KronBlur."""

    def __init__(self, A):
        self.A = sp.csr_matrix(A)

    def matvec(self, x):
        return self.A @ x

    def rmatvec(self, y):
        return self.A.T @ y

    def right(self, Pv, Ph) -> "SparseOp":
        return SparseOp(self.A @ sp.kron(Ph, Pv, format="csr"))

    def explicit(self):
        return self.A


def colsumsq(op) -> np.ndarray:
    """Column sums of squares of A_k (the paper's diag(A_k^T A_k))."""
    if isinstance(op, KronBlur):
        cv = np.asarray(op.Av.multiply(op.Av).sum(axis=0)).ravel()
        ch = np.asarray(op.Ah.multiply(op.Ah).sum(axis=0)).ravel()
        return np.kron(ch, cv)
    A = sp.csr_matrix(op.explicit())
    return np.asarray(A.multiply(A).sum(axis=0)).ravel()


class Hierarchy:
    """One-sided multigrid hierarchy for one outer weighting D (lambda-free).

    A: KronBlur (deblurring) or SparseOp (tomography) forward operator.
    M: sparse D L (2n x n).  levels >= 1; level 0 is the finest.
    """

    def __init__(self, A, M, nv: int, nh: int, levels: int, periodic: bool):
        self.levels = levels
        self.nv = [nv >> k for k in range(levels)]
        self.nh = [nh >> k for k in range(levels)]
        if any(v << k != nv for k, v in enumerate(self.nv)) or \
           any(h << k != nh for k, h in enumerate(self.nh)):
            raise ValueError("grid not divisible by 2^(levels-1)")
        self.Pv, self.Ph, self.P = [], [], []
        for k in range(levels - 1):
            Pv = interpolation_1d(self.nv[k], periodic)
            Ph = interpolation_1d(self.nh[k], periodic)
            self.Pv.append(Pv)
            self.Ph.append(Ph)
            self.P.append(sp.kron(Ph, Pv, format="csr"))
        self.A = [A]
        self.M = [sp.csr_matrix(M)]
        for k in range(levels - 1):
            self.A.append(self.A[k].right(self.Pv[k], self.Ph[k]))
            self.M.append((self.M[k] @ self.P[k]).tocsr())
        self.diagA = [colsumsq(a) for a in self.A]
        self.diagM = [np.asarray(m.multiply(m).sum(axis=0)).ravel()
                      for m in self.M]
        # Gershgorin row sums |A_k^T A_k| 1 (A_k >= 0 entrywise) and |M_k^T M_k| 1
        self.rowabsA, self.rowabsM = [], []
        for k in range(levels):
            ones = np.ones(self.nv[k] * self.nh[k])
            self.rowabsA.append(self.A[k].rmatvec(self.A[k].matvec(ones)))
            S = (self.M[k].T @ self.M[k]).tocsr()
            self.rowabsM.append(np.asarray(abs(S).sum(axis=1)).ravel())

    # -- level operators ------------------------------------------------
    def K(self, k: int, lam: float, x):
        a = self.A[k]
        return a.rmatvec(a.matvec(x)) + lam * lam * (self.M[k].T @ (self.M[k] @ x))

    def diag(self, k: int, lam: float):
        return self.diagA[k] + lam * lam * self.diagM[k]

    def gershgorin(self, k: int, lam: float) -> float:
        return float(np.max((self.rowabsA[k] + lam * lam * self.rowabsM[k])
                            / self.diag(k, lam)))

    def coarse_matrix(self, lam: float) -> np.ndarray:
        k = self.levels - 1
        Ak = np.asarray(sp.csr_matrix(self.A[k].explicit()).toarray())
        Mk = self.M[k].toarray()
        return Ak.T @ Ak + lam * lam * (Mk.T @ Mk)


def chebyshev(K, dinv, b, x, a: float, bnd: float, steps: int):
    """`steps` Chebyshev iterations for K x = b preconditioned by diag^-1,
    targeting the interval [a, bnd] of the scaled spectrum (three-term
    recurrence in the form of Adams, Brezina, Hu and Tuminaro, 2003).

    x may be None for a zero initial guess.
    """
    theta = 0.5 * (bnd + a)
    delta = 0.5 * (bnd - a)
    sigma = theta / delta
    rho_old = 1.0 / sigma
    r = b.copy() if x is None else b - K(x)
    d = dinv * r / theta
    x = d.copy() if x is None else x + d
    for _ in range(1, steps):
        r = b - K(x)
        rho = 1.0 / (2.0 * sigma - rho_old)
        d = rho * rho_old * d + (2.0 * rho / delta) * dinv * r
        x = x + d
        rho_old = rho
    return x


class VCycle:
    """z = M^{-1} r by one V(nu, nu) cycle (Algorithm 1, gamma = 1).

    nu and ratio may be given per level (sequences indexed by level, finest
    first); a scalar applies to every level.
    """

    def __init__(self, H: Hierarchy, lam: float, nu=2, ratio=4.0):
        self.H, self.lam = H, lam
        L = H.levels
        self.nu = list(nu) if hasattr(nu, "__len__") else [nu] * L
        self.ratio = list(ratio) if hasattr(ratio, "__len__") else [ratio] * L
        self.dinv = [1.0 / H.diag(k, lam) for k in range(H.levels)]
        self.rho = [H.gershgorin(k, lam) for k in range(H.levels)]
        self.chol = sla.cho_factor(H.coarse_matrix(lam), lower=True)

    def cycle(self, b, k: int = 0):
        H, lam = self.H, self.lam
        if k == H.levels - 1:
            return sla.cho_solve(self.chol, b)
        K = lambda v: H.K(k, lam, v)
        lo, hi = self.rho[k] / self.ratio[k], self.rho[k]
        x = chebyshev(K, self.dinv[k], b, None, lo, hi, self.nu[k])
        res = b - K(x)
        e = self.cycle(H.P[k].T @ res, k + 1)
        x = x + H.P[k] @ e
        return chebyshev(K, self.dinv[k], b, x, lo, hi, self.nu[k])

    __call__ = cycle


def cg_relax(K, dinv, b, x, steps: int):
    """`steps` iterations of CG preconditioned by diag^-1 on K x = b from x
    (None for zero): the relaxation of the paper's Section 3.2 (diagonally
    preconditioned CG on every level, restarted at each relaxation)."""
    x = np.zeros_like(b) if x is None else np.array(x, dtype=np.float64)
    r = b - K(x)
    z = dinv * r
    p = z.copy()
    gamma = float(r @ z)
    for i in range(steps):
        if gamma == 0.0:
            break
        q = K(p)
        alpha = gamma / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        if i + 1 < steps:
            z = dinv * r
            gnew = float(r @ z)
            p = z + (gnew / gamma) * p
            gamma = gnew
    return x


class KrylovVCycle:
    """z ~ M^{-1} r by one V(nu_pre, nu_post) cycle whose relaxation on every
    level but the coarsest is diagonally preconditioned CG (Section 3.2: two
    pre- and one post-relaxation sweep, one CG iteration per sweep), with
    the exact coarsest solve of Algorithm 1.  The CG coefficients depend on
    the residual, so the cycle is not a fixed linear map: it belongs under
    a flexible outer method (the paper uses FGMRES)."""

    def __init__(self, H: Hierarchy, lam: float, nu_pre=2, nu_post=1):
        self.H, self.lam = H, lam
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.dinv = [1.0 / H.diag(k, lam) for k in range(H.levels)]
        self.chol = sla.cho_factor(H.coarse_matrix(lam), lower=True)

    def cycle(self, b, k: int = 0):
        H, lam = self.H, self.lam
        if k == H.levels - 1:
            return sla.cho_solve(self.chol, b)
        K = lambda v: H.K(k, lam, v)
        x = cg_relax(K, self.dinv[k], b, None, self.nu_pre)
        res = b - K(x)
        e = self.cycle(H.P[k].T @ res, k + 1)
        x = x + H.P[k] @ e
        return cg_relax(K, self.dinv[k], b, x, self.nu_post)

    __call__ = cycle
