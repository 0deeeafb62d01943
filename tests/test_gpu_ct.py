"""Tomography (sparse A) path against the oracle.

The projector is generated once on the CPU and handed to both sides.  On
the GPU the one-sided hierarchy A_{k+1} = A_k P and every A_k^T are built
by the library; the level operators K_k(lambda) must match the oracle's
SciPy products to relative 1e-12, the FP32 V-cycle the oracle's FP64
V-cycle to single-precision accuracy (3e-5 of the largest entry, as for the
deblurring path), and the sweep solutions the oracle's dense solves to
relative 1e-6 (FP64 PCG with the FP32 V-cycle, relative residual 1e-13).
"""
import numpy as np
import pytest

from oracle.pcg import CtOracle
from tests.gpu_util import dev, host
from workloads.ct import small_ct

pytestmark = pytest.mark.gpu


def _prob(P, ell, levels, nu=2, ratio=4.0):
    from paper_2306_11067_amd import TomographyProblem
    return TomographyProblem(P.rowptr, P.col, P.val, P.N, levels, nu=nu,
                             cheb_ratio=ratio, weights=dev(P.weights[ell]))


@pytest.fixture(scope="module")
def case():
    P = small_ct(32, 24, 3, 4)
    return P, _prob(P, 1, 3), CtOracle(P.matrix(), P.N, P.lbc, P.weights[1], 3)


def test_ct_forward_adjoint_match_scipy(case):
    P, prob, O = case
    rng = np.random.default_rng(1)
    A = P.matrix()
    x = rng.standard_normal(2 * P.n)
    y = rng.standard_normal(2 * P.m)
    ax = host(prob.forward(dev(x), nvec=2))
    aty = host(prob.adjoint(dev(y), nvec=2))
    for s in range(2):
        want = A @ x[s * P.n:(s + 1) * P.n]
        np.testing.assert_allclose(ax[s * P.m:(s + 1) * P.m], want, rtol=0,
                                   atol=1e-12 * np.abs(want).max())
        want = A.T @ y[s * P.m:(s + 1) * P.m]
        np.testing.assert_allclose(aty[s * P.n:(s + 1) * P.n], want, rtol=0,
                                   atol=1e-12 * np.abs(want).max())


def test_ct_grouped_products_equal_single_products(case):
    """Products over several vectors take the kernel that reads each row of
    A once for a group of vectors; it sums in the same order as the
    one-vector kernel, so every vector's result is bitwise the same as
    computing it alone (and equals SciPy's within rounding)."""
    P, prob, O = case
    rng = np.random.default_rng(2)
    k = 9                                   # one group of 8, one of 1
    x = rng.standard_normal(k * P.n)
    y = rng.standard_normal(k * P.m)
    ax = host(prob.forward(dev(x), nvec=k))
    aty = host(prob.adjoint(dev(y), nvec=k))
    for s in range(k):
        one = host(prob.forward(dev(x[s * P.n:(s + 1) * P.n]), nvec=1))
        assert np.array_equal(ax[s * P.m:(s + 1) * P.m], one), s
        one = host(prob.adjoint(dev(y[s * P.m:(s + 1) * P.m]), nvec=1))
        assert np.array_equal(aty[s * P.n:(s + 1) * P.n], one), s


def test_ct_level_operators_match_oracle(case):
    P, prob, O = case
    H = O.H
    rng = np.random.default_rng(2)
    lams = np.array([1e-3, 0.3, 40.0])
    for k in range(H.levels):
        nk = H.nv[k] * H.nh[k]
        v = rng.standard_normal(len(lams) * nk)
        got = host(prob.apply_normal(k, lams, dev(v))).reshape(len(lams), nk)
        for s, lam in enumerate(lams):
            want = H.K(k, lam, v[s * nk:(s + 1) * nk])
            err = np.abs(got[s] - want).max() / np.abs(want).max()
            assert err < 1e-12, (k, lam, err)


def test_ct_gershgorin_matches_oracle(case):
    P, prob, O = case
    H = O.H
    lams = np.array([1e-3, 0.1, 10.0])
    for k in range(H.levels):
        got = prob.gershgorin(k, lams)
        want = np.array([H.gershgorin(k, lam) for lam in lams])
        np.testing.assert_allclose(got, want, rtol=1e-12)


def test_ct_fp32_vcycle_close_to_oracle(case):
    P, prob, O = case
    rng = np.random.default_rng(3)
    lams = np.array([1e-3, 0.3, 40.0])
    r = rng.standard_normal(len(lams) * P.n)
    got = host(prob.vcycle(lams, dev(r))).reshape(len(lams), P.n)
    for s, lam in enumerate(lams):
        want = O.vcycle(lam, nu=2, ratio=4.0)(r[s * P.n:(s + 1) * P.n])
        err = np.abs(got[s] - want).max() / np.abs(want).max()
        assert 0.0 < err < 3e-5, (lam, err)


@pytest.mark.parametrize("ell", [0, 1])
def test_ct_sweep_matches_oracle(ell):
    P = small_ct(64, 48, 4, 5)
    prob = _prob(P, ell, 4, nu=4, ratio=16.0)
    # the edge-weighted system reaches an error/residual ratio ~1e6 at
    # lambda = 1e-3, so the residual target is 1e-13
    x, res, sem, info = prob.solve_sweep(dev(P.b), P.lams, 1e-13, poll_every=8)
    x = host(x)
    O = CtOracle(P.matrix(), P.N, P.lbc, P.weights[ell], 4)
    for s, lam in enumerate(P.lams):
        xr, rel = O.reference(P.b, lam)
        assert rel < 1e-11
        e = np.linalg.norm(x[s] - xr) / np.linalg.norm(xr)
        assert e <= 1e-6, (ell, lam, e, info[s])
        rho, eta = O.pair(xr, P.b)
        assert abs(res[s] - rho) <= 1e-6 * rho and abs(sem[s] - eta) <= 1e-6 * eta
        assert info[s]["flags"] & 1, info[s]


def test_ct_full_size_properties():
    # The 256 x 256 parallel-beam workload (180 angles, 363 bins, 1.5e7
    # nonzeros) with the benchmark's smoothing on three lambdas of its
    # sweep.  No closed form exists at this size, so the oracle checks what
    # holds at any size: its own FP64 residual of the normal equations at the
    # GPU's x (<= the tolerance, up to rounding) and the L-curve pair.
    import bench
    from workloads.ct import config3
    P = config3()
    lams = np.array([1e-1, 3.0, 100.0])
    prob = _prob(P, 1, P.levels, nu=bench.NU_FINE, ratio=bench.RATIO_FINE)
    tol = 1e-12
    x, res, sem, info = prob.solve_sweep(dev(P.b), lams, tol, poll_every=16)
    x = host(x)
    O = CtOracle(P.matrix(), P.N, P.lbc, P.weights[1], 1)
    f = O.rhs(P.b)
    for s, lam in enumerate(lams):
        assert info[s]["flags"] & 1, info[s]
        r = f - O.K(lam)(x[s])
        rel = np.linalg.norm(r) / np.linalg.norm(f)
        assert rel <= 1.05 * tol, (lam, rel)
        rho, eta = O.pair(x[s], P.b)
        assert abs(res[s] - rho) <= 1e-10 * rho and abs(sem[s] - eta) <= 1e-10 * eta
