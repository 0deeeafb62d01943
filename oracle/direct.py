"""Direct solutions of the regularized problem (FP64).

Each routine computes x*(lambda) = argmin ||A x - b||^2 + lambda^2 ||D L x||^2
(Section 1, eq. (LSreg)), by a different route:

  solve_dense    -- Cholesky of K = A^T A + lambda^2 L^T D^2 L (eq. (normal))
  solve_stacked  -- least squares on [A; lambda D L] x = [b; 0] (eq. (LStall)),
                    which never forms the normal matrix
  solve_fft      -- periodic blur and periodic gradient with D = I: K is
                    block-circulant, diagonalized by the 2D DFT
  solve_dct      -- half-sample reflective blur (symmetric taps) with the
                    Neumann gradient and D = I: diagonalized by the DCT-II
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

from . import operators as ops


def solve_dense(A, M, b, lam: float) -> np.ndarray:
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    M = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    K = A.T @ A + lam * lam * (M.T @ M)
    c = sla.cho_factor(K, lower=True)
    return sla.cho_solve(c, A.T @ b)


def solve_stacked(A, M, b, lam: float) -> np.ndarray:
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    M = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    S = np.vstack([A, lam * M])
    rhs = np.concatenate([b, np.zeros(M.shape[0])])
    return np.linalg.lstsq(S, rhs, rcond=None)[0]


def _circulant_symbol(taps, n):
    """DFT of the first column of the circulant blur (B x)_i = sum t_k x_{i-k}."""
    r = (len(taps) - 1) // 2
    c = np.zeros(n)
    for k in range(-r, r + 1):
        c[k % n] += taps[k + r]
    return np.fft.fft(c)


def solve_fft(taps_v, taps_h, nv, nh, b, lam: float) -> np.ndarray:
    """Closed form for periodic A and periodic L, D = I.

    With a = DFT symbol of A, the normal matrix has eigenvalues
    |a|^2 + lambda^2 (|e^{iw_v} - 1|^2 + |e^{iw_h} - 1|^2) and A^T b has
    coefficients conj(a) * DFT(b).
    """
    av = _circulant_symbol(taps_v, nv)
    ah = _circulant_symbol(taps_h, nh)
    a = ah[:, None] * av[None, :]                 # [j, i] layout
    wv = 2 * np.pi * np.arange(nv) / nv
    wh = 2 * np.pi * np.arange(nh) / nh
    lap = (2 - 2 * np.cos(wh))[:, None] + (2 - 2 * np.cos(wv))[None, :]
    B = np.fft.fft2(np.asarray(b).reshape(nh, nv))
    X = np.conj(a) * B / (np.abs(a) ** 2 + lam * lam * lap)
    return np.real(np.fft.ifft2(X)).ravel()


def reflective_symbol(taps, n):
    """Eigenvalues of the half-sample reflective blur with symmetric taps in
    the orthonormal DCT-II basis: t_0 + 2 sum_k t_k cos(pi j k / n)."""
    r = (len(taps) - 1) // 2
    j = np.arange(n)
    s = np.full(n, taps[r], dtype=np.float64)
    for k in range(1, r + 1):
        s += 2 * taps[r + k] * np.cos(np.pi * j * k / n)
    return s


def solve_dct(taps_v, taps_h, nv, nh, b, lam: float) -> np.ndarray:
    """Closed form for reflective A (symmetric taps), Neumann L, D = I.

    The Neumann difference Laplacian L_v^T L_v has DCT-II eigenvalues
    2 - 2 cos(pi j / n).
    """
    av = reflective_symbol(taps_v, nv)
    ah = reflective_symbol(taps_h, nh)
    a = ah[:, None] * av[None, :]
    lap = (2 - 2 * np.cos(np.pi * np.arange(nh) / nh))[:, None] + \
          (2 - 2 * np.cos(np.pi * np.arange(nv) / nv))[None, :]
    B = sfft.dctn(np.asarray(b).reshape(nh, nv), type=2, norm="ortho")
    X = a * B / (a * a + lam * lam * lap)
    return sfft.idctn(X, type=2, norm="ortho").ravel()


def spectral_inverse(taps_v, taps_h, nv, nh, bc, lbc, lam: float):
    """Exact inverse of K0 = A^T A + lambda^2 L^T L (D = I) as a function,
    for the matching boundary pairs (periodic, periodic) and
    (reflective, neumann).  Used as a preconditioner for D != I."""
    if bc == "periodic" and lbc == "periodic":
        av = _circulant_symbol(taps_v, nv)
        ah = _circulant_symbol(taps_h, nh)
        a2 = np.abs(ah[:, None] * av[None, :]) ** 2
        wv = 2 * np.pi * np.arange(nv) / nv
        wh = 2 * np.pi * np.arange(nh) / nh
        lap = (2 - 2 * np.cos(wh))[:, None] + (2 - 2 * np.cos(wv))[None, :]
        den = a2 + lam * lam * lap

        def apply(r):
            R = np.fft.fft2(np.asarray(r).reshape(nh, nv))
            return np.real(np.fft.ifft2(R / den)).ravel()
        return apply
    if bc == "reflective" and lbc == "neumann":
        av = reflective_symbol(taps_v, nv)
        ah = reflective_symbol(taps_h, nh)
        a = ah[:, None] * av[None, :]
        lap = (2 - 2 * np.cos(np.pi * np.arange(nh) / nh))[:, None] + \
              (2 - 2 * np.cos(np.pi * np.arange(nv) / nv))[None, :]
        den = a * a + lam * lam * lap

        def apply(r):
            R = sfft.dctn(np.asarray(r).reshape(nh, nv), type=2, norm="ortho")
            return sfft.idctn(R / den, type=2, norm="ortho").ravel()
        return apply
    raise ValueError("no spectral inverse for this boundary pair")


def normal_rhs(A, b):
    return A.T @ b


__all__ = ["solve_dense", "solve_stacked", "solve_fft", "solve_dct",
           "spectral_inverse", "reflective_symbol", "ops"]
