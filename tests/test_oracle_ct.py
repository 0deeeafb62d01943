"""Pins of the tomography inputs and of the oracle with a sparse projector.

The projector is an input (generated once, handed to both the oracle and
the GPU path); it is pinned against closed forms of the geometry.  The
oracle's normal equations with a general sparse A are pinned against a
dense Cholesky solve, and its V-cycle-preconditioned CG against both.
"""
import math

import numpy as np
import pytest

from oracle.multigrid import Hierarchy, SparseOp
from oracle.pcg import CtOracle, pcg
from workloads.ct import parallel_beam, small_ct


def _chord(th, s, N):
    """Length of the line x cos(th) + y sin(th) = s inside [-N/2, N/2]^2."""
    c, sn = math.cos(th), math.sin(th)
    h = N / 2.0
    pts = []
    if abs(sn) > 1e-15:
        for x in (-h, h):
            y = (s - x * c) / sn
            if -h - 1e-12 <= y <= h + 1e-12:
                pts.append((x, y))
    if abs(c) > 1e-15:
        for y in (-h, h):
            x = (s - y * sn) / c
            if -h - 1e-12 <= x <= h + 1e-12:
                pts.append((x, y))
    if len(pts) < 2:
        return 0.0
    return max(math.dist(p, q) for p in pts for q in pts)


@pytest.mark.parametrize("N,na,nb", [(16, 12, 23), (32, 24, 46), (24, 18, 35)])
def test_row_lengths_are_chords(N, na, nb):
    rp, ci, va = parallel_beam(N, na, nb)
    s = np.arange(nb) - (nb - 1) / 2.0
    for k in range(na):
        th = k * math.pi / na
        for b in range(nb):
            row = k * nb + b
            L = va[rp[row]:rp[row + 1]].astype(np.float64).sum()
            want = _chord(th, s[b], N)
            axis = abs(math.sin(th)) < 1e-12 or abs(math.cos(th)) < 1e-12
            if axis and abs(abs(s[b]) - N / 2) < 1e-12:
                want *= 0.5   # on the outer edge: the other half is outside
            assert abs(L - want) <= 4e-6 * max(1.0, L), (k, b)


def test_rows_sorted_and_in_range():
    N = 24
    rp, ci, va = parallel_beam(N, 18, 35)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0)
    assert ci.min() >= 0 and ci.max() < N * N
    assert np.all(va > 0)
    for r in range(len(rp) - 1):
        c = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(c) > 0)


def test_transpose_symmetry():
    # Swapping x and y maps angle k to angle n_angles/2 - k (theta -> pi/2 -
    # theta) with the same offset: A_k applied to the transposed image
    # equals A_{n/2-k} applied to the image.
    N, na, nb = 24, 18, 35
    rp, ci, va = parallel_beam(N, na, nb)
    import scipy.sparse as sp
    A = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(na * nb, N * N))
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, N * N)
    xt = x.reshape(N, N).T.ravel()     # p = i + N j  ->  swap i and j
    y, yt = A @ x, A @ xt
    for k in range(na // 2 + 1):
        a = yt[k * nb:(k + 1) * nb]
        bb = y[(na // 2 - k) * nb:(na // 2 - k + 1) * nb]
        assert np.abs(a - bb).max() <= 1e-5 * np.abs(bb).max(), k


def test_axis_aligned_ray_on_grid_line_splits():
    # theta = 0 with an even N and an odd bin count puts every ray on a
    # vertical grid line: each of its N row segments is shared half/half.
    N, nb = 8, 11
    rp, ci, va = parallel_beam(N, 4, nb)
    b = (nb - 1) // 2            # s = 0: the line x = 0 between columns 3, 4
    row = slice(rp[b], rp[b + 1])
    cols = ci[row]
    assert len(cols) == 2 * N
    np.testing.assert_allclose(va[row], 0.5)
    assert set(cols // N) == {N // 2 - 1, N // 2}


def _ct_oracle(P, ell, levels):
    return CtOracle(P.matrix(), P.N, P.lbc, P.weights[ell], levels)


def test_ct_problem_data_is_projection_plus_noise():
    P = small_ct(32, 24, 3, 4)
    b_true = P.matrix() @ P.x_true
    noise = P.b - b_true
    np.testing.assert_allclose(np.linalg.norm(noise),
                               P.noise * np.linalg.norm(b_true), rtol=1e-12)


@pytest.mark.parametrize("ell", [0, 1])
def test_ct_mg_pcg_reaches_dense_solution(ell):
    P = small_ct(32, 24, 3, 4)
    O = _ct_oracle(P, ell, 3)
    for lam in (1e-2, 1.0, 30.0):
        xd, rel = O.reference(P.b, lam)
        assert rel < 1e-11
        x, it, _, _ = O.mg_pcg(P.b, lam, tol=1e-13)
        assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd), (lam, it)


def test_ct_one_sided_hierarchy_is_galerkin():
    # A_{k+1}^T A_{k+1} = P^T A_k^T A_k P for the sparse projector.
    P = small_ct(32, 24, 3, 4)
    O = _ct_oracle(P, 1, 3)
    H = O.H
    for k in range(2):
        G = (H.A[k].explicit().T @ H.A[k].explicit()).toarray()
        Pk = H.P[k].toarray()
        Gc = (H.A[k + 1].explicit().T @ H.A[k + 1].explicit()).toarray()
        np.testing.assert_allclose(Gc, Pk.T @ G @ Pk, atol=1e-10 * np.abs(G).max())
