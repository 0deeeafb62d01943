"""Pins for the oracle of the paper's own preconditioner: the V(2,1) cycle
with diagonally preconditioned CG relaxation (Section 3.2), run under
flexible PCG.  Checked against properties of CG and of Galerkin multigrid
rather than against itself."""
import numpy as np

import workloads as W
from oracle.multigrid import Hierarchy, KrylovVCycle, cg_relax
from oracle.pcg import DeblurOracle


def _spd(n, seed, spread=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    K = Q @ np.diag(np.logspace(0, np.log10(spread), n)) @ Q.T
    return 0.5 * (K + K.T)


def _knorm(K, e):
    return float(np.sqrt(e @ (K @ e)))


def test_cg_relax_terminates_after_about_n_steps():
    # exact arithmetic: the solution after n steps; in floating point CG's
    # finite termination is delayed by a step or two (plain CG on the same
    # matrix behaves alike), so n + 3 steps reach the rounding level
    n = 12
    K = _spd(n, 1)
    dinv = 1.0 / np.diag(K)
    b = np.random.default_rng(2).standard_normal(n)
    x = cg_relax(lambda v: K @ v, dinv, b, None, n + 3)
    xs = np.linalg.solve(K, b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_cg_relax_one_step_exact_when_k_is_a_multiple_of_its_diagonal():
    rng = np.random.default_rng(3)
    d = rng.uniform(0.5, 4.0, 20)
    K = 3.5 * np.diag(d)
    b = rng.standard_normal(20)
    x = cg_relax(lambda v: K @ v, 1.0 / np.diag(K), b, None, 1)
    assert np.allclose(x, b / (3.5 * d), rtol=1e-14, atol=0)


def test_cg_relax_energy_error_never_grows():
    n = 30
    K = _spd(n, 4, spread=1e5)
    dinv = 1.0 / np.diag(K)
    b = np.random.default_rng(5).standard_normal(n)
    xs = np.linalg.solve(K, b)
    errs = [_knorm(K, xs - cg_relax(lambda v: K @ v, dinv, b, None, s))
            for s in range(0, 12)]
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(11)), errs


def test_cg_relax_from_a_start_equals_relaxing_the_residual_equation():
    n = 25
    K = _spd(n, 6)
    dinv = 1.0 / np.diag(K)
    rng = np.random.default_rng(7)
    b, x0 = rng.standard_normal(n), rng.standard_normal(n)
    a = cg_relax(lambda v: K @ v, dinv, b, x0, 3)
    c = x0 + cg_relax(lambda v: K @ v, dinv, b - K @ x0, None, 3)
    assert np.allclose(a, c, rtol=1e-12, atol=1e-12)


def _problem(levels):
    P = W.small_deblur(32, 32, 2, 1.0, "reflective", "neumann", levels,
                       nlam=3)
    return P, DeblurOracle(P.nv, P.nh, P.taps_v, P.taps_h, P.bc, P.lbc,
                           P.weights[1], levels)


def test_one_level_cycle_is_the_exact_solve():
    P, O = _problem(1)
    lam = 1e-2
    b = np.random.default_rng(8).standard_normal(P.nv * P.nh)
    z = KrylovVCycle(O.H, lam)(b)
    Kd = O.H.coarse_matrix(lam)
    assert np.allclose(z, np.linalg.solve(Kd, b), rtol=1e-10, atol=1e-12)


def test_cycle_never_increases_the_energy_error():
    # Galerkin coarse operators and CG relaxations: as an iteration
    # x <- x + V(b - K x) the cycle cannot increase the K-norm error; a sign
    # error in the correction or a transposed interpolation breaks this
    P, O = _problem(3)
    rng = np.random.default_rng(9)
    for lam in (1e-4, 1e-2, 1.0):
        K = O.K(lam)
        V = KrylovVCycle(O.H, lam, 2, 1)
        for _ in range(3):
            xs = rng.standard_normal(P.nv * P.nh)
            after = xs - V(K(xs))            # error after one cycle from 0
            ka = float(np.sqrt(after @ K(after)))
            kb = float(np.sqrt(xs @ K(xs)))
            assert ka < kb, (lam, ka, kb)


def test_flexible_pcg_with_the_cycle_reaches_the_reference():
    P, O = _problem(3)
    for lam in (1e-3, 1e-1):
        xr, _ = O.reference(P.b, lam)
        x, its, _, _ = O.krylov_mg_pcg(P.b, lam, tol=1e-11, maxit=20000)
        assert np.linalg.norm(x - xr) <= 1e-7 * np.linalg.norm(xr), (lam, its)
