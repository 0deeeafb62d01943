"""The outer reweighting loop (Algorithm 2) on the GPU against the oracle.

  * rls_update_weights (eq. (g)) on Neumann and periodic grids, with D = I
    and with stored weights, for q = 1, 2 and 0.7, on a grid whose 2n
    gradient entries are not a whole number of 256-thread blocks and on a
    512 x 512 grid (more blocks than the maximum pass launches, so its
    grid-stride loop runs): the new weights within 1e-13 absolute of the
    oracle's (the oracle forms D L as a sparse product, -d x_k + d x_{k+1},
    the kernel d (x_{k+1} - x_k): a few FP64 roundings of the entry, divided
    by ||D L x||_inf, which is of the order of the entries here), and
    ||D L x||_inf within 1e-14 relative;
  * a flat image leaves D bitwise unchanged and reports ||D L x||_inf = 0;
  * two updates in a row match the oracle's chain;
  * rls_regularize on a 64 x 64 reflective deblurring problem with 16
    lambdas in [1e-4, 1] and q = 2: the same index at every outer iteration
    and the same stop as the oracle's Algorithm 2 with exact solves, the
    returned solution within 1e-6 of the oracle's, and the final weights
    within 1e-6 (each update sees a solution with the solver's error);
  * rls_regularize on a 32 x 32 tomography problem (24 angles, 12 lambdas
    in [1e-3, 1e2], FP32 V-cycle under FP64 PCG), six outer iterations: the
    same choices as the oracle's dense solves (the closest call among them
    has the nearest point 11 % nearer to the corner than the next), solution
    and weights within 1e-6.
"""
import numpy as np
import pytest

import workloads as W
from oracle import outer
from oracle.pcg import CtOracle, DeblurOracle
from tests.gpu_util import dev, host
from workloads.ct import small_ct

pytestmark = pytest.mark.gpu

GRIDS = {
    # name: (nv, nh, lbc, bc, levels)
    "neumann92x76": (92, 76, "neumann", "reflective", 3),
    "periodic64x48": (64, 48, "periodic", "periodic", 3),
    "neumann512": (512, 512, "neumann", "reflective", 5),
}


def _problem(nv, nh, lbc, bc, levels, d=None):
    from paper_2306_11067_amd import Problem
    taps = W.gaussian_taps(2, 1.0)
    return Problem(nv, nh, taps, taps, bc, lbc, levels,
                   weights=None if d is None else dev(d))


def _image(nv, nh, rng):
    i = np.arange(nv)[None, :]
    j = np.arange(nh)[:, None]
    smooth = np.sin(2 * np.pi * i / nv) * np.cos(2 * np.pi * j / nh)
    return (smooth + 0.3 * rng.standard_normal((nh, nv))).ravel()


@pytest.mark.parametrize("q", [1.0, 2.0, 0.7])
@pytest.mark.parametrize("unit", [True, False])
@pytest.mark.parametrize("name", list(GRIDS))
def test_weight_update_matches_oracle(name, unit, q):
    nv, nh, lbc, bc, levels = GRIDS[name]
    rng = np.random.default_rng(31)
    n = nv * nh
    d0 = np.ones(2 * n) if unit else rng.uniform(0.01, 1.0, 2 * n)
    P = _problem(nv, nh, lbc, bc, levels, None if unit else d0)
    x = _image(nv, nh, rng)
    top = P.update_weights(dev(x), q)
    got = host(P.weights())
    want, wtop = outer.weight_update(d0, x, nv, nh, lbc, q)
    assert abs(top - wtop) <= 1e-14 * wtop, (top, wtop)
    err = np.abs(got - want).max()
    assert err <= 1e-13, (name, unit, q, err)
    assert np.count_nonzero(got == 0.0) >= 1
    P.close()


def test_flat_image_keeps_weights_bitwise():
    nv, nh, lbc, bc, levels = GRIDS["neumann92x76"]
    d0 = np.random.default_rng(2).uniform(0.01, 1.0, 2 * nv * nh)
    P = _problem(nv, nh, lbc, bc, levels, d0)
    top = P.update_weights(dev(np.full(nv * nh, 0.25)), 2.0)
    assert top == 0.0
    assert np.array_equal(host(P.weights()), d0)
    P.close()


def test_two_updates_match_oracle_chain():
    nv, nh, lbc, bc, levels = GRIDS["periodic64x48"]
    rng = np.random.default_rng(4)
    P = _problem(nv, nh, lbc, bc, levels)
    d = np.ones(2 * nv * nh)
    for q in (2.0, 1.0):
        x = _image(nv, nh, rng)
        P.update_weights(dev(x), q)
        d, _ = outer.weight_update(d, x, nv, nh, lbc, q)
    assert np.abs(host(P.weights()) - d).max() <= 1e-13
    P.close()


def test_regularize_matches_oracle_algorithm():
    from paper_2306_11067_amd import Problem
    P_ = W.small_deblur(64, 64, 3, 1.5, "reflective", "neumann", 3, nlam=16)
    q, maxouter = 2.0, 12
    n = P_.nv * P_.nh

    def make(d):
        return DeblurOracle(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                            np.ones(2 * n) if d is None else d, 1)

    xw, chosen_w, dw, stopped_w = outer.regularize(
        make, P_.b, P_.lams, q, maxouter, P_.nv, P_.nh, P_.lbc)
    prob = Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                   P_.levels)
    x, chosen, info = prob.regularize(dev(P_.b), P_.lams, q, 1e-12,
                                      maxouter=maxouter)
    assert chosen == chosen_w, (chosen, chosen_w)
    assert info["stopped"] == stopped_w
    assert info["chosen_index"] == chosen_w[-1]
    xg = host(x)
    assert np.linalg.norm(xg - xw) <= 1e-6 * np.linalg.norm(xw)
    dg = host(prob.weights())
    dref = np.ones(2 * n) if dw is None else dw
    assert np.abs(dg - dref).max() <= 1e-6
    prob.close()


def test_regularize_tomography_matches_oracle_algorithm():
    from paper_2306_11067_amd import TomographyProblem
    P = small_ct(32, 24, 3, 12)
    A = P.matrix()
    q, maxouter = 2.0, 6
    n = P.N * P.N

    def make(d):
        return CtOracle(A, P.N, P.lbc, np.ones(2 * n) if d is None else d, 1)

    xw, chosen_w, dw, stopped_w = outer.regularize(
        make, P.b, P.lams, q, maxouter, P.N, P.N, P.lbc)
    prob = TomographyProblem(P.rowptr, P.col, P.val, P.N, 3, nu=4,
                             cheb_ratio=16.0)
    x, chosen, info = prob.regularize(dev(P.b), P.lams, q, 1e-13,
                                      maxouter=maxouter, poll_every=8)
    assert chosen == chosen_w, (chosen, chosen_w)
    assert info["stopped"] == stopped_w
    xg = host(x)
    assert np.linalg.norm(xg - xw) <= 1e-6 * np.linalg.norm(xw)
    dref = np.ones(2 * n) if dw is None else dw
    assert np.abs(host(prob.weights()) - dref).max() <= 1e-6
    prob.close()


def test_outer_argument_errors():
    from paper_2306_11067_amd import RLSError
    from paper_2306_11067_amd import _lib as L
    P_ = W.small_deblur(64, 64, 3, 1.5, "reflective", "neumann", 3, nlam=12)
    prob = _problem(64, 64, "neumann", "reflective", 3)
    b = dev(P_.b)
    bad = [
        (P_.lams[:9], 2.0, 5),                      # fewer than 10 lambdas
        (P_.lams[::-1], 2.0, 5),                    # decreasing
        (np.r_[P_.lams[:5], P_.lams[4:11]], 2.0, 5),  # repeated value
        (P_.lams, 0.0, 5),                          # q <= 0
        (P_.lams, np.nan, 5),
        (P_.lams, 2.0, 0),                          # no outer iteration
    ]
    for lams, q, mo in bad:
        with pytest.raises(RLSError) as e:
            prob.regularize(b, lams, q, 1e-10, maxouter=mo)
        assert e.value.status == L.RLS_E_ARG, (lams, q, mo)
    for q in (0.0, -1.0, np.inf):
        with pytest.raises(RLSError) as e:
            prob.update_weights(dev(P_.b), q)
        assert e.value.status == L.RLS_E_ARG
    # the problem is still usable after the rejected calls
    assert np.array_equal(host(prob.weights()), np.ones(2 * 64 * 64))
    prob.close()


def test_regularize_one_outer_iteration_and_ten_lambdas():
    # maxouter = 1: one full sweep, the corner of its own L-curve, no
    # weight update; m = 10: every pruned window is the whole grid
    from paper_2306_11067_amd import Problem, lcurve_corner
    P_ = W.small_deblur(64, 64, 3, 1.5, "reflective", "neumann", 3, nlam=10)
    prob = Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                   P_.levels)
    b = dev(P_.b)
    x, chosen, info = prob.regularize(b, P_.lams, 2.0, 1e-12, maxouter=1)
    assert info["outer"] == 1 and not info["stopped"]
    assert np.array_equal(host(prob.weights()), np.ones(2 * P_.nv * P_.nh))
    xs, res, sem, _ = prob.solve_sweep(b, P_.lams, 1e-12)
    assert chosen == [lcurve_corner(P_.lams, res, sem)]
    xr = host(xs[chosen[0]])
    assert np.linalg.norm(host(x) - xr) <= 1e-12 * np.linalg.norm(xr)
    n = P_.nv * P_.nh

    def make(d):
        return DeblurOracle(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                            np.ones(2 * n) if d is None else d, 1)

    _, chosen_w, _, stopped_w = outer.regularize(
        make, P_.b, P_.lams, 2.0, 6, P_.nv, P_.nh, P_.lbc)
    _, chosen6, info6 = prob.regularize(b, P_.lams, 2.0, 1e-12, maxouter=6)
    assert chosen6 == chosen_w and info6["stopped"] == stopped_w
    prob.close()
