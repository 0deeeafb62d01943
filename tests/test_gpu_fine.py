"""The tiled finest-level Chebyshev kernel (band radius fixed at compile time).

The finest-level smoothing step takes this kernel when the grid is a whole
number of 64 x 16 tiles and both Gram bands are uniform (periodic, or
reflective with a symmetric PSF); otherwise the general level-operator
kernel.  Checked on the same seeded inputs:
  * the V-cycle around it against the oracle's V-cycle (FP64 bar 1e-10 of
    the largest entry plus 4 u kappa, u = 2^-53 and kappa the condition
    number of the coarsest-level matrix, whose direct solve passes its
    rounding on with that gain: the 21 x 21 PSF at lambda = 1e-4 has kappa
    8e7 and both fine kernels sit 1.7e-9 from the oracle there, 3e-16 from
    each other; FP32 V-cycle 3e-5, the bars of the general kernel);
  * against the same V-cycle with the general kernel forced through
    RLS_FINE_KERNEL=generic: equal up to rounding (FP64 1e-12), and not
    bit-identical, which shows that the two problems ran different kernels
    (the tiled kernel adds symmetric tap pairs before multiplying);
  * a sweep that uses it against the oracle's x*(lambda) (bar 1e-6);
  * launches with one slot take 512-thread workgroups, more slots 256-thread
    ones, with the same arithmetic per output and the same order of the
    per-tile dot partials: a V-cycle on one lambda equals that lambda's slot
    of a three-lambda V-cycle bitwise (and batched sweeps equal single-lambda
    sweeps, tested with the sweeps).
The cases cover band radii 2, 8 (padded from 6 in the other direction), 14
(the 15 x 15 PSF of the 512 x 512 workload) and 20 (the 21 x 21 PSF of the
2048 x 2048 configuration), several tile rows and
columns, both index maps, and four smoothing steps per level so that the
kernel runs five times per V-cycle.
"""
import numpy as np
import pytest

import workloads as W
from oracle.pcg import DeblurOracle
from tests.gpu_util import dev, host
from tests.test_gpu_sweep import _check_against_reference

pytestmark = pytest.mark.gpu

CASES = {
    # name: (nv, nh, r_v, r_h, sigma, bc, lbc, levels)
    "reflective128x64_r7": (128, 64, 7, 7, 3.0, "reflective", "neumann", 3),
    "periodic64x48_r4r3": (64, 48, 4, 3, 2.0, "periodic", "periodic", 3),
    "reflective64x32_r1": (64, 32, 1, 1, 0.8, "reflective", "neumann", 2),
    "reflective192x128_r8": (192, 128, 8, 8, 3.0, "reflective", "neumann", 4),
    "reflective128x64_r10": (128, 64, 10, 10, 4.0, "reflective", "neumann", 3),
}
NU = 4
RATIO = 4.0


def _setup(name, precision="fp64", generic=False, monkeypatch=None):
    from paper_2306_11067_amd import Problem
    nv, nh, rv, rh, sg, bc, lbc, levels = CASES[name]
    rng = np.random.default_rng(7)
    tv = W.gaussian_taps(rv, sg)
    th = W.gaussian_taps(rh, sg * 0.9)
    d = rng.uniform(0.01, 1.0, 2 * nv * nh)
    if generic:
        monkeypatch.setenv("RLS_FINE_KERNEL", "generic")
    try:
        P = Problem(nv, nh, tv, th, bc, lbc, levels, nu=NU, cheb_ratio=RATIO,
                    weights=dev(d), precision=precision)
    finally:
        if generic:
            monkeypatch.delenv("RLS_FINE_KERNEL")
    O = DeblurOracle(nv, nh, tv, th, bc, lbc, d, levels)
    return P, O, rng


def _vcycles(P, n, rng, lams):
    r = rng.standard_normal(len(lams) * n)
    return r, host(P.vcycle(lams, dev(r))).reshape(len(lams), n)


LAMS = np.array([1e-4, 1e-2, 1.0])


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_tiled_vcycle_matches_oracle(name, precision):
    P, O, rng = _setup(name, precision)
    n = O.nv * O.nh
    r, got = _vcycles(P, n, rng, LAMS)
    for s, lam in enumerate(LAMS):
        if precision == "fp64":
            kappa = np.linalg.cond(O.H.coarse_matrix(lam))
            bar = 1e-10 + 4 * 2.0 ** -53 * kappa
        else:
            bar = 3e-5
        want = O.vcycle(lam, nu=NU, ratio=RATIO)(r[s * n:(s + 1) * n])
        err = np.abs(got[s] - want).max() / np.abs(want).max()
        assert err < bar, (name, precision, lam, err, bar)


@pytest.mark.parametrize("name", list(CASES))
def test_tiled_vcycle_matches_general_kernel(name, monkeypatch):
    P, O, _ = _setup(name)
    G, _, _ = _setup(name, generic=True, monkeypatch=monkeypatch)
    n = O.nv * O.nh
    r = np.random.default_rng(11).standard_normal(len(LAMS) * n)
    a = host(P.vcycle(LAMS, dev(r))).reshape(len(LAMS), n)
    b = host(G.vcycle(LAMS, dev(r))).reshape(len(LAMS), n)
    diff = np.abs(a - b).max() / np.abs(b).max()
    assert diff < 1e-12, (name, diff)
    assert diff > 0.0, name


@pytest.mark.parametrize("name", list(CASES))
def test_tiled_variants_agree_bitwise(name):
    P, O, _ = _setup(name)
    n = O.nv * O.nh
    r = np.random.default_rng(12).standard_normal(len(LAMS) * n)
    batch = host(P.vcycle(LAMS, dev(r))).reshape(len(LAMS), n)
    for s in range(len(LAMS)):
        one = host(P.vcycle(LAMS[s:s + 1], dev(r[s * n:(s + 1) * n])))
        assert np.array_equal(one, batch[s]), (name, s)


def test_tiled_sweep_matches_oracle():
    import torch
    from paper_2306_11067_amd import Problem
    P_ = W.small_deblur(128, 64, 7, 3.0, "reflective", "neumann", 3, nlam=4)
    prob = Problem(P_.nv, P_.nh, P_.taps_v, P_.taps_h, P_.bc, P_.lbc,
                   P_.levels, nu=NU, cheb_ratio=RATIO,
                   weights=dev(P_.weights[1]))
    x, res, sem, info = prob.solve_sweep(dev(P_.b), P_.lams, 1e-12,
                                         poll_every=8)
    torch.cuda.synchronize()
    n = P_.nv * P_.nh
    _check_against_reference(P_, 1, host(x).reshape(len(P_.lams), n), res,
                             sem, info)
