"""The paper's second workloads on the GPU against the oracle.

  * The deblurring problem of the paper's Section 4.6 on a 64 x 64 grid:
    zero-boundary (Toeplitz) Kronecker blur with anisotropic truncated
    Gaussians (radius 6, sigma 1.25 along the contiguous axis; radius 7,
    sigma 1.5 across), Neumann gradient, 30 lambdas in [1e-3, 1e2].  Sweeps
    with D = I and with the edge weighting: at every fifth lambda and the
    largest, x and both L-curve norms within 1e-6 of the oracle's x* (CG to
    the FP64 floor).  Algorithm 2 (q = 2, five outer iterations) makes the
    oracle's choices (the closest call has the nearest point 7 % nearer to
    the corner sample than the next).
  * Limited-angle tomography as in the paper's Section 4.5 (66 angles 0, 2,
    ..., 130 degrees, 91 bins, 64 x 64 pixels, 12 lambdas in [1e-3, 1e2]),
    FP32 V-cycle under FP64 PCG: sweeps with both weightings against the
    oracle's dense solves at every second lambda, 1e-6.
"""
import numpy as np
import pytest

import bench
import workloads as W
from oracle import outer
from oracle.pcg import CtOracle, DeblurOracle
from tests.gpu_util import dev, host
from workloads.ct import limited_angle_ct

pytestmark = pytest.mark.gpu

BAR = 1e-6
TOL = 1e-13


def _deblur_problem(P, d=None):
    from paper_2306_11067_amd import Problem
    return Problem(P.nv, P.nh, P.taps_v, P.taps_h, P.bc, P.lbc, P.levels,
                   nu=bench.NU_FINE, cheb_ratio=bench.RATIO_FINE,
                   nu_coarse=bench.NU_COARSE,
                   cheb_ratio_coarse=bench.RATIO_COARSE,
                   weights=None if d is None else dev(d))


def _check(O, b, lams, idx, x, res, sem, info):
    for s in idx:
        xr, rel = O.reference(b, lams[s])
        assert rel < 1e-10, (s, rel)
        e = np.linalg.norm(x[s] - xr) / np.linalg.norm(xr)
        assert e <= BAR, (s, lams[s], e, info[s])
        rho, eta = O.pair(xr, b)
        assert abs(res[s] - rho) <= BAR * rho, (s, res[s], rho)
        assert abs(sem[s] - eta) <= BAR * eta, (s, sem[s], eta)
        assert info[s]["flags"] & 1, info[s]


@pytest.mark.parametrize("ell", [0, 1])
def test_paper_deblur_sweep_matches_oracle(ell):
    P = W.paper_deblur(64)
    d = P.weights[ell]
    prob = _deblur_problem(P, d)
    x, res, sem, info = prob.solve_sweep(dev(P.b), P.lams, TOL, poll_every=16)
    x = host(x)
    prob.close()
    O = DeblurOracle(P.nv, P.nh, P.taps_v, P.taps_h, P.bc, P.lbc, d, 1)
    idx = list(range(0, len(P.lams), 5)) + [len(P.lams) - 1]
    _check(O, P.b, P.lams, idx, x, res, sem, info)


def test_paper_deblur_regularize_matches_oracle_algorithm():
    P = W.paper_deblur(64)
    n = P.nv * P.nh
    q, maxouter = 2.0, 5

    def make(d):
        return DeblurOracle(P.nv, P.nh, P.taps_v, P.taps_h, P.bc, P.lbc,
                            np.ones(2 * n) if d is None else d, 1)

    xw, chosen_w, dw, stopped_w = outer.regularize(
        make, P.b, P.lams, q, maxouter, P.nv, P.nh, P.lbc)
    prob = _deblur_problem(P)
    x, chosen, info = prob.regularize(dev(P.b), P.lams, q, TOL,
                                      maxouter=maxouter, poll_every=16)
    assert chosen == chosen_w, (chosen, chosen_w)
    assert info["stopped"] == stopped_w
    assert np.linalg.norm(host(x) - xw) <= BAR * np.linalg.norm(xw)
    prob.close()


@pytest.mark.parametrize("ell", [0, 1])
def test_limited_angle_ct_sweep_matches_oracle(ell):
    from paper_2306_11067_amd import TomographyProblem
    C = limited_angle_ct(64, nlam=12)
    prob = TomographyProblem(C.rowptr, C.col, C.val, C.N, C.levels, nu=4,
                             cheb_ratio=16.0, weights=dev(C.weights[ell]))
    x, res, sem, info = prob.solve_sweep(dev(C.b), C.lams, TOL, poll_every=8)
    x = host(x)
    prob.close()
    O = CtOracle(C.matrix(), C.N, C.lbc, C.weights[ell], 1)
    _check(O, C.b, C.lams, range(0, len(C.lams), 2), x, res, sem, info)
