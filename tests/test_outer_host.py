"""The library's host-side steps of Algorithm 2 against the oracle, on the
CPU: rls_lcurve_corner (natural splines of the log-log L-curve, largest
curvature, nearest point) and rls_trim_window (the pruned range of Section
3.4), plus their argument checks.  Neither touches a GPU.

Corner parity is exact (an index): the two sides evaluate the same splines
with different rounding, so the cases are chosen with the nearest point at
least 1.5x closer to the corner sample than the next one (a near-tie could
legitimately go either way).
"""
import numpy as np
import pytest

from oracle import outer
from tests.test_oracle_outer import _tikhonov_curve


def _lib():
    from paper_2306_11067_amd import _lib as L
    return L


def _curves():
    k = np.arange(1, 201, dtype=float)
    rng = np.random.default_rng(21)
    out = []
    for decay in (0.7, 1.0, 1.5, 2.0):
        for noise in (1e-4, 1e-3, 1e-2):
            for nlam in (10, 16, 30, 64):
                s = k ** -decay * np.exp(-k / 20)
                beta = s * k ** -0.5 + noise * rng.standard_normal(k.size)
                lam = np.logspace(-6, 0, nlam)
                rho, eta = _tikhonov_curve(lam, s, beta)
                out.append((lam, rho, eta))
    return out


def _margin(lam, rho, eta):
    _, xs, ys, kappa = outer.lcurve_curvature(lam, rho, eta)
    k = int(np.argmax(kappa))
    d2 = (np.log10(rho) - xs[k]) ** 2 + (np.log10(eta) - ys[k]) ** 2
    s = np.sort(d2)
    return s[1] / max(s[0], 1e-300)


def test_corner_matches_oracle():
    from paper_2306_11067_amd import lcurve_corner
    checked = 0
    for lam, rho, eta in _curves():
        if _margin(lam, rho, eta) < 1.5:
            continue
        assert lcurve_corner(lam, rho, eta) == \
            outer.lcurve_corner(lam, rho, eta), len(lam)
        checked += 1
    assert checked >= 30, checked


def test_corner_two_legs_and_minimum_size():
    from paper_2306_11067_amd import lcurve_corner
    lam = np.logspace(-3, 1, 21)
    j = 8
    idx = np.arange(21)
    X = np.where(idx <= j, 0.0, 0.25 * (idx - j))
    Y = np.where(idx <= j, 0.25 * (j - idx), 0.0)
    assert lcurve_corner(lam, 10.0 ** X, 10.0 ** Y) == j
    # three points: the middle one of a right angle
    assert lcurve_corner([1e-2, 1e-1, 1.0], [1.0, 1.0, 10.0],
                         [10.0, 1.0, 1.0]) == 1


def test_trim_window_matches_oracle():
    from paper_2306_11067_amd import trim_window
    for m in (10, 11, 20, 64):
        for i in range(m):
            assert trim_window(i, m) == outer.trim_window(i, m), (i, m)


@pytest.mark.parametrize("lam,rho,eta", [
    ([1e-2, 1e-1], [1.0, 2.0], [2.0, 1.0]),                 # m < 3
    ([1e-2, 1e-2, 1.0], [1.0, 2.0, 3.0], [3.0, 2.0, 1.0]),  # not increasing
    ([1e-2, 1e-1, 1.0], [1.0, 0.0, 3.0], [3.0, 2.0, 1.0]),  # zero residual
    ([1e-2, 1e-1, 1.0], [1.0, 2.0, 3.0], [3.0, np.nan, 1.0]),
    ([-1e-2, 1e-1, 1.0], [1.0, 2.0, 3.0], [3.0, 2.0, 1.0]),
])
def test_corner_rejects_bad_input(lam, rho, eta):
    from paper_2306_11067_amd import RLSError, lcurve_corner
    with pytest.raises(RLSError) as e:
        lcurve_corner(lam, rho, eta)
    assert e.value.status == _lib().RLS_E_ARG


@pytest.mark.parametrize("i,m", [(0, 9), (-1, 20), (20, 20)])
def test_trim_window_rejects_bad_input(i, m):
    from paper_2306_11067_amd import RLSError, trim_window
    with pytest.raises(RLSError) as e:
        trim_window(i, m)
    assert e.value.status == _lib().RLS_E_ARG
