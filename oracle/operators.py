"""Explicit operators of the regularized least-squares problem (FP64).

Vectorization follows the paper's Section 2: an n_v x n_h image is stored
column-major, pixel (i, j) at index i + n_v*j, i the vertical index.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _ext(j: int, n: int, bc: str):
    """Index of the pixel that supplies position j of the extended signal."""
    if 0 <= j < n:
        return j
    if bc == "periodic":
        return j % n
    if bc == "reflective":          # half-sample symmetric: x[-1] = x[0]
        m = j % (2 * n)
        return m if m < n else 2 * n - 1 - m
    return None                     # zero boundary: outside pixels are 0


def blur_matrix_1d(taps, n: int, bc: str) -> sp.csr_matrix:
    """1D blur B with (B x)_i = sum_k t_k x_ext(i - k), k = -r..r.

    The deblurring operator of the paper (Section 4.6) is a Kronecker product
    of two such 1D matrices; there the boundary is zero (a plain Toeplitz
    matrix).  Periodic and half-sample reflective boundaries are also given.
    """
    taps = np.asarray(taps, dtype=np.float64)
    r = (len(taps) - 1) // 2
    rows, cols, vals = [], [], []
    for i in range(n):
        for k in range(-r, r + 1):
            c = _ext(i - k, n, bc)
            if c is None:
                continue
            rows.append(i)
            cols.append(c)
            vals.append(taps[k + r])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))  # duplicates add


def blur_matrix(taps_v, taps_h, nv: int, nh: int, bc: str) -> sp.csr_matrix:
    """2D separable blur A = A_h (x) A_v (Kronecker product, Section 4.6)."""
    return sp.kron(blur_matrix_1d(taps_h, nh, bc),
                   blur_matrix_1d(taps_v, nv, bc), format="csr")


def difference_1d(n: int, lbc: str) -> sp.csr_matrix:
    """Forward difference with one row per pixel (Section 2, eq. (gradient)).

    Rows 0..n-2 are the paper's L_v (-1 on the diagonal, +1 above it).  The
    last row is zero for the paper's (Neumann) gradient -- a padding row that
    leaves L^T D^2 L unchanged -- or the wrap-around difference x_0 - x_{n-1}
    for a periodic gradient.
    """
    rows = list(range(n - 1)) * 2
    cols = list(range(n - 1)) + list(range(1, n))
    vals = [-1.0] * (n - 1) + [1.0] * (n - 1)
    if lbc == "periodic":
        rows += [n - 1, n - 1]
        cols += [n - 1, 0]
        vals += [-1.0, 1.0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def gradient(nv: int, nh: int, lbc: str) -> sp.csr_matrix:
    """L = [I (x) L_v ; L_h (x) I] (Section 2, eq. (gradient)), 2n x n.

    The first n rows are vertical differences, the next n horizontal ones,
    each plane indexed like the image (i + n_v*j).
    """
    Lv = difference_1d(nv, lbc)
    Lh = difference_1d(nh, lbc)
    return sp.vstack([sp.kron(sp.identity(nh), Lv),
                      sp.kron(Lh, sp.identity(nv))], format="csr")


def regularizer(d, nv: int, nh: int, lbc: str) -> sp.csr_matrix:
    """M = D L with D = diag(d) over both gradient planes (Section 1, eq. (ml))."""
    return (sp.diags(np.asarray(d, float)) @ gradient(nv, nh, lbc)).tocsr()


def normal_matrix(A, M, lam: float) -> sp.csr_matrix:
    """K(lambda) = A^T A + lambda^2 M^T M (Section 3.2, eq. (normal))."""
    return (A.T @ A + (lam * lam) * (M.T @ M)).tocsr()


class KronBlur:
    """A = A_h (x) A_v applied through the identity (B (x) C) vec(X) =
    vec(C X B^T), for grids too large for an explicit Kronecker matrix."""

    def __init__(self, Av, Ah):
        self.Av = sp.csr_matrix(Av)
        self.Ah = sp.csr_matrix(Ah)
        self.nv_out, self.nv = self.Av.shape
        self.nh_out, self.nh = self.Ah.shape

    def matvec(self, x):
        X = np.asarray(x).reshape(self.nh, self.nv).T          # X[i, j]
        Y = self.Ah @ (self.Av @ X).T                           # (Av X Ah^T)^T
        return np.asarray(Y).ravel()

    def rmatvec(self, y):
        Y = np.asarray(y).reshape(self.nh_out, self.nv_out).T
        X = self.Ah.T @ (self.Av.T @ Y).T
        return np.asarray(X).ravel()

    def right(self, Pv, Ph) -> "KronBlur":
        """One-sided coarsening A P with P = P_h (x) P_v."""
        return KronBlur(self.Av @ Pv, self.Ah @ Ph)

    def explicit(self) -> sp.csr_matrix:
        return sp.kron(self.Ah, self.Av, format="csr")


def lcurve_pair(A_apply, M, x, b):
    """(||A x - b||_2, ||M x||_2): one point of the L-curve (Section 1)."""
    return (float(np.linalg.norm(A_apply(x) - b)),
            float(np.linalg.norm(M @ x)))
