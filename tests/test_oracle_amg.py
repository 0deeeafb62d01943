"""Pins for the Ruge-Stueben AMG oracle (paper Sections 3.1 and 3.2): a
hand-worked 1D case, the strength rule on a hand-made row, properties that
classical coarsening guarantees for zero-row-sum M-matrices, and the
hierarchy under both V-cycles."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import operators as ops
from oracle.amg import (AmgHierarchy, rs_interpolation, rs_split,
                        strong_connections)
from oracle.multigrid import KrylovVCycle, VCycle
from oracle.pcg import DeblurOracle, pcg


def test_strength_rule_on_a_hand_made_row():
    # row 0: -1, -0.3, -0.2 off the diagonal; theta * max = 0.25, so the
    # -1 and -0.3 couplings are strong and -0.2 is not
    K = sp.csr_matrix(np.array([[1.5, -1.0, -0.3, -0.2],
                                [-1.0, 1.0, 0.0, 0.0],
                                [-0.3, 0.0, 0.3, 0.0],
                                [-0.2, 0.0, 0.0, 0.2]]))
    S = strong_connections(K, 0.25).toarray()
    assert list(S[0]) == [0, 1, 1, 0]


def test_one_dimensional_laplacian_by_hand():
    # Neumann 1D Laplacian on 9 points (all couplings equal, all strong).
    # Greedy pass: point 1 (two dependants, lowest index) is C and makes 0
    # and 2 F, which raises point 3's measure; then 3, 5, 7 follow the same
    # way.  Interpolation: end points copy their C neighbour, interior F
    # points average their two C neighbours.
    L = ops.difference_1d(9, "neumann")
    K = (L.T @ L).tocsr()
    is_c, _ = rs_split(K)
    assert list(np.nonzero(is_c)[0]) == [1, 3, 5, 7]
    P = rs_interpolation(K).toarray()
    want = np.zeros((9, 4))
    want[0, 0] = 1.0
    for c, i in enumerate([1, 3, 5, 7]):
        want[i, c] = 1.0
    for i, (a, b) in zip([2, 4, 6], [(0, 1), (1, 2), (2, 3)]):
        want[i, a] = want[i, b] = 0.5
    want[8, 3] = 1.0
    assert np.allclose(P, want, rtol=0, atol=1e-15)


def _weighted_laplacian(nv, nh, seed):
    d = np.random.default_rng(seed).uniform(0.01, 1.0, 2 * nv * nh)
    M = ops.regularizer(d, nv, nh, "neumann")
    return (M.T @ M).tocsr()


def test_zero_row_sum_properties():
    for seed, (nv, nh) in ((1, (12, 10)), (2, (16, 16))):
        K = _weighted_laplacian(nv, nh, seed)
        is_c, S = rs_split(K)
        P = rs_interpolation(K)
        # constants are interpolated exactly (zero row sums)
        assert np.allclose(P @ np.ones(P.shape[1]), 1.0, rtol=0, atol=1e-12)
        # every strong F-F connection shares a strong C point
        for i in np.nonzero(~is_c)[0]:
            Si = set(S.indices[S.indptr[i]:S.indptr[i + 1]])
            Ci = {j for j in Si if is_c[j]}
            for j in Si:
                if not is_c[j]:
                    Sj = set(S.indices[S.indptr[j]:S.indptr[j + 1]])
                    assert Sj & Ci, (i, j)
        # Galerkin operator: symmetric, zero row sums, fewer unknowns
        Kc = (P.T @ K @ P).toarray()
        assert np.allclose(Kc, Kc.T, atol=1e-13)
        assert np.allclose(Kc @ np.ones(Kc.shape[0]), 0.0, atol=1e-12)
        assert 0 < P.shape[1] < P.shape[0]


def _amg_problem():
    P = W.small_deblur(32, 32, 2, 1.0, "reflective", "neumann", 3, nlam=3)
    O = DeblurOracle(P.nv, P.nh, P.taps_v, P.taps_h, P.bc, P.lbc,
                     P.weights[1], 1)
    H = AmgHierarchy(O.A, O.M, levels=4, max_coarse=200)
    return P, O, H


def test_amg_cycles_reduce_the_energy_error_and_precondition_pcg():
    P, O, H = _amg_problem()
    assert H.levels >= 3 and H.A[-1].A.shape[1] <= 200
    rng = np.random.default_rng(4)
    for lam in (1e-3, 1e-1):
        K = O.K(lam)
        V = KrylovVCycle(H, lam, 2, 1)
        xs = rng.standard_normal(P.nv * P.nh)
        after = xs - V(K(xs))
        assert after @ K(after) < xs @ K(xs), lam
        xr, _ = O.reference(P.b, lam)
        Vc = VCycle(H, lam, nu=2, ratio=4.0)
        x, its, _, _ = pcg(K, O.rhs(P.b), Vc, tol=1e-11, maxit=20000)
        assert np.linalg.norm(x - xr) <= 1e-7 * np.linalg.norm(xr), (lam, its)


def test_amg_hierarchy_on_a_tomography_operator():
    # the hierarchy only needs A explicitly: the same construction serves a
    # sparse projector (one-sided A_{k+1} = A_k P_k)
    from oracle.pcg import CtOracle
    from workloads.ct import small_ct
    C = small_ct(32, 24, 3, 3)
    O = CtOracle(C.matrix(), C.N, C.lbc, C.weights[1], 1)
    H = AmgHierarchy(O.A, O.M, levels=4, max_coarse=200)
    assert H.levels >= 3
    for lam in (1e-2, 1.0):
        K = O.K(lam)
        xr, _ = O.reference(C.b, lam)
        x, its, _, _ = pcg(K, O.rhs(C.b), VCycle(H, lam, nu=2, ratio=4.0),
                           tol=1e-12, maxit=20000)
        assert np.linalg.norm(x - xr) <= 1e-7 * np.linalg.norm(xr), (lam, its)
