"""Full-sweep parity of the HIP path (rls_solve_sweep) against the oracle.

x_i is compared with the oracle's x*(lambda_i) computed to the FP64 floor
(DFT / DCT closed forms for D = I, otherwise CG preconditioned by the exact
D = I inverse).  Bar: relative error <= 1e-6 in x and in the L-curve pair,
with the GPU run at a relative residual tolerance of 1e-12 (residual 1e-8
leaves errors near 1e-3 at the smallest lambda: the error/residual ratio of
these systems reaches ~1e5).  Iteration counts are compared with the
oracle's own V-cycle-preconditioned CG at equal tolerance.
"""
import numpy as np
import pytest

import workloads as W
from oracle.pcg import DeblurOracle
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _problem(P_, ell):
    from paper_2306_11067_amd import Problem
    return Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                   P_.levels, nu=2, cheb_ratio=4.0,
                   weights=dev(P_.weights[ell]))


def _check_against_reference(P_, ell, x, res, sem, info, tol_err=1e-6):
    O = DeblurOracle(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                     P_.weights[ell], P_.levels)
    for s, lam in enumerate(P_.lams):
        xr, rel = O.reference(P_.b, lam)
        assert rel < 1e-11
        e = np.linalg.norm(x[s] - xr) / np.linalg.norm(xr)
        assert e <= tol_err, (ell, lam, e, info[s])
        rho, eta = O.pair(xr, P_.b)
        assert abs(res[s] - rho) <= tol_err * rho, (lam, res[s], rho)
        assert abs(sem[s] - eta) <= tol_err * eta, (lam, sem[s], eta)
        assert info[s]["flags"] & 1, info[s]
        assert info[s]["relres_true"] < 1e-11, info[s]


@pytest.mark.parametrize("ell", [0, 1])
def test_config1_sweep_matches_oracle(ell):
    P_ = W.config1()
    prob = _problem(P_, ell)
    x, res, sem, info = prob.solve_sweep(dev(P_.b), P_.lams, 1e-12)
    _check_against_reference(P_, ell, host(x), res, sem, info)


def test_reflective_sweep_matches_oracle():
    P_ = W.small_deblur(128, 96, 3, 1.5, "reflective", "neumann", 3, nlam=6,
                        outer=1)
    prob = _problem(P_, 1)
    x, res, sem, info = prob.solve_sweep(dev(P_.b), P_.lams, 1e-12)
    _check_against_reference(P_, 1, host(x), res, sem, info)


def test_iteration_counts_match_oracle_mg_pcg():
    P_ = W.config1()
    prob = _problem(P_, 1)
    lams = P_.lams[4:]
    tol = 1e-10
    _, _, _, info = prob.solve_sweep(dev(P_.b), lams, tol)
    O = DeblurOracle(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                     P_.weights[1], P_.levels)
    for s, lam in enumerate(lams):
        _, it, _, _ = O.mg_pcg(P_.b, lam, tol=tol)
        assert abs(info[s]["iters"] - it) <= 1, (lam, info[s]["iters"], it)


def test_batched_equals_individual_and_is_deterministic():
    P_ = W.small_deblur(64, 64, 2, 1.0, "reflective", "neumann", 3, nlam=4)
    prob = _problem(P_, 1)
    b = dev(P_.b)
    xb, rb, sb, ib = prob.solve_sweep(b, P_.lams, 1e-10)
    xb = host(xb)
    xb2 = host(prob.solve_sweep(b, P_.lams, 1e-10)[0])
    assert np.array_equal(xb, xb2)
    for s, lam in enumerate(P_.lams):
        xs, rs, ss, is_ = prob.solve_sweep(b, [lam], 1e-10)
        assert np.array_equal(host(xs)[0], xb[s])
        assert is_[0]["iters"] == ib[s]["iters"]


def test_warm_start_and_maxit_flags():
    P_ = W.small_deblur(64, 64, 2, 1.0, "reflective", "neumann", 3, nlam=3)
    prob = _problem(P_, 1)
    b = dev(P_.b)
    x, _, _, info = prob.solve_sweep(b, P_.lams, 1e-10)
    # restarting from the solution: converged at once
    x2, _, _, info2 = prob.solve_sweep(b, P_.lams, 1e-9, x0=x.reshape(-1))
    assert all(i["iters"] <= 1 for i in info2), info2
    # iteration cap
    _, _, _, info3 = prob.solve_sweep(b, P_.lams, 1e-14, maxit=2)
    assert all(i["flags"] & 2 and i["iters"] == 2 for i in info3), info3


def test_weights_change_between_sweeps():
    P_ = W.small_deblur(64, 64, 2, 1.0, "reflective", "neumann", 3, nlam=2)
    prob = _problem(P_, 0)
    b = dev(P_.b)
    prob.set_weights(dev(P_.weights[1]))
    x1 = host(prob.solve_sweep(b, P_.lams, 1e-12)[0])
    fresh = _problem(P_, 1)
    x2 = host(fresh.solve_sweep(b, P_.lams, 1e-12)[0])
    assert np.array_equal(x1, x2)


def test_error_paths():
    from paper_2306_11067_amd import RLSError
    P_ = W.small_deblur(32, 32, 2, 1.0, "reflective", "neumann", 2, nlam=2)
    prob = _problem(P_, 0)
    b = dev(P_.b)
    with pytest.raises(RLSError) as e:
        prob.solve_sweep(b, [0.0, 1.0], 1e-8)
    assert e.value.status == -1
    with pytest.raises(RLSError) as e:
        prob.solve_sweep(b, [1.0], -1.0)
    assert e.value.status == -1
    bad = P_.weights[1].copy()
    bad[5] = -0.5
    with pytest.raises(RLSError) as e:
        prob.set_weights(dev(bad))
    assert e.value.status == -1
    bad[5] = np.nan
    with pytest.raises(RLSError):
        prob.set_weights(dev(bad))


def test_graph_replay_equals_direct_launches():
    # The same sweep with iteration chunks replayed as HIP graphs and with
    # kernels launched one by one gives bitwise identical results, twice.
    P_ = W.small_deblur(96, 64, 3, 1.5, "reflective", "neumann", 3, nlam=5)
    prob = _problem(P_, 1)
    b = dev(P_.b)
    xd, rd, sd, idd = prob.solve_sweep(b, P_.lams, 1e-11, graph=False,
                                       poll_every=6)
    for _ in range(2):
        xg, rg, sg, ig = prob.solve_sweep(b, P_.lams, 1e-11, graph=True,
                                          poll_every=6)
        assert np.array_equal(host(xg), host(xd))
        assert [i["iters"] for i in ig] == [i["iters"] for i in idd]
        assert np.array_equal(rg, rd) and np.array_equal(sg, sd)


def test_kernel_timer_counts_finest_smoothing_launches():
    # With the timer on, every finest-level Chebyshev-step launch is timed;
    # results are bitwise those of the graph-replayed sweep, and the bytes
    # follow the per-launch model n * (40 * active + 24).
    from paper_2306_11067_amd import Problem
    P_ = W.small_deblur(128, 96, 3, 1.5, "reflective", "neumann", 3, nlam=3)
    nu = 5
    prob = Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                   P_.levels, nu=nu, cheb_ratio=30.0, nu_coarse=2,
                   cheb_ratio_coarse=4.0, weights=dev(P_.weights[1]))
    b = dev(P_.b)
    x0, _, _, i0 = prob.solve_sweep(b, P_.lams, 1e-10)
    prob.kernel_timer(True)
    x1, _, _, i1 = prob.solve_sweep(b, P_.lams, 1e-10, poll_every=4)
    launches, seconds, nbytes = prob.kernel_timer_read()
    prob.kernel_timer(False)
    assert np.array_equal(host(x0), host(x1))
    n = P_.nv * P_.nh
    cycles = [i["iters"] + 1 for i in i1]     # gate passes + initial cycle
    assert launches >= max(cycles) * (2 * nu - 3)
    assert seconds > 0
    lo = n * 40.0 * (2 * nu - 3) * sum(cycles) * 0.5
    hi = n * (40.0 * len(cycles) + 24.0) * launches
    assert lo <= nbytes <= hi, (lo, nbytes, hi)
