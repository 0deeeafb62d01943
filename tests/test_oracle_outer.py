"""Pins for the oracle of the outer loop (Algorithm 2): eq. (g), the L-curve
corner, the trimming window and the stopping rule, checked against values
fixed by hand, closed forms and invariants rather than against themselves.
"""
import numpy as np
import pytest

from oracle import outer


# ---- eq. (g) --------------------------------------------------------------

def test_weights_constant_image_leave_d_unchanged():
    # D L x = 0: the paper's extreme case, D stays as it was
    rng = np.random.default_rng(0)
    d = rng.uniform(0.1, 1.0, 2 * 6 * 5)
    for lbc in ("neumann", "periodic"):
        dn, top = outer.weight_update(d, np.full(30, 3.0), 6, 5, lbc, 1.0)
        assert top == 0.0
        assert np.array_equal(dn, d)


def test_weights_two_step_image_by_hand():
    # 4 x 3 image (nv = 4 rows along the contiguous axis, nh = 3 columns):
    # column 0 = 0, column 1 = 1, column 2 = 1.5.  Vertical differences are
    # zero; horizontal differences: 1 between columns 0 and 1, 0.5 between
    # 1 and 2, and 0 in the Neumann padding column.  With D = I and q = 2:
    # g = 1 and 0.5, so d = 0 and 0.75 there and 1 elsewhere.
    nv, nh = 4, 3
    x = np.repeat([0.0, 1.0, 1.5], nv)
    dn, top = outer.weight_update(np.ones(2 * nv * nh), x, nv, nh, "neumann",
                                  2.0)
    assert top == 1.0
    want = np.ones(2 * nv * nh)
    want[nv * nh + 0:nv * nh + 4] = 0.0        # horizontal plane, column 0
    want[nv * nh + 4:nv * nh + 8] = 0.75       # column 1
    assert np.array_equal(dn, want)


def test_weights_use_the_current_weights_in_g():
    # the same image with D = 0.5 on the jump between columns 0 and 1:
    # |D L x| is 0.5 on both jumps, so g = 1 on both and both get d = 0
    # (g taken from |L x| alone would give 0.75 on the second jump)
    nv, nh = 4, 3
    x = np.repeat([0.0, 1.0, 1.5], nv)
    d0 = np.ones(2 * nv * nh)
    d0[nv * nh + 0:nv * nh + 4] = 0.5
    dn, top = outer.weight_update(d0, x, nv, nh, "neumann", 2.0)
    assert top == 0.5
    want = np.ones(2 * nv * nh)
    want[nv * nh + 0:nv * nh + 8] = 0.0
    assert np.array_equal(dn, want)


def test_weights_periodic_wrap_jump_is_largest():
    # a ramp 0..5 along the contiguous axis, periodic: the wrap-around
    # difference (0 - 5) is the largest, so only the last row gets d = 0
    nv, nh = 6, 2
    x = np.tile(np.arange(nv, dtype=float), nh)
    dn, top = outer.weight_update(np.ones(2 * nv * nh), x, nv, nh,
                                  "periodic", 1.0)
    assert top == 5.0
    v = dn[:nv * nh].reshape(nh, nv)
    assert np.array_equal(v[:, :nv - 1], np.full((nh, nv - 1), 0.8))
    assert np.array_equal(v[:, nv - 1], np.zeros(nh))
    assert np.array_equal(dn[nv * nh:], np.ones(nv * nh))


def test_weights_invariants():
    rng = np.random.default_rng(1)
    nv, nh = 9, 7
    d = rng.uniform(0.01, 1.0, 2 * nv * nh)
    x = rng.standard_normal(nv * nh)
    for q in (0.5, 1.0, 3.0):
        dn, top = outer.weight_update(d, x, nv, nh, "neumann", q)
        assert np.all(dn >= 0.0) and np.all(dn <= d)        # 0 <= d(l) <= 1
        dn2, top2 = outer.weight_update(d, 7.5 * x, nv, nh, "neumann", q)
        assert np.allclose(dn2, dn, rtol=1e-14, atol=1e-16)  # scale-free
        assert np.isclose(top2, 7.5 * top, rtol=1e-14)
        assert np.count_nonzero(dn == 0.0) >= 1              # the max entry


# ---- L-curve corner -------------------------------------------------------

def _tikhonov_curve(lam, s, beta):
    """Residual and seminorm of min ||diag(s) x - beta||^2 + lam^2 ||x||^2
    (closed form through the SVD)."""
    lam = np.asarray(lam)[:, None]
    f = s * s / (s * s + lam * lam)
    rho = np.sqrt(np.sum(((1 - f) * beta) ** 2, axis=1))
    eta = np.sqrt(np.sum((f * beta / s) ** 2, axis=1))
    return rho, eta


def _true_corner(s, beta, lo, hi):
    # largest curvature of the exact curve, from finite differences on a
    # very fine log-lambda grid (no spline involved)
    t = np.linspace(lo, hi, 200001)
    rho, eta = _tikhonov_curve(10.0 ** t, s, beta)
    X, Y = np.log10(rho), np.log10(eta)
    h = t[1] - t[0]
    x1, y1 = np.gradient(X, h), np.gradient(Y, h)
    x2, y2 = np.gradient(x1, h), np.gradient(y1, h)
    k = (x1 * y2 - y1 * x2) / (x1 * x1 + y1 * y1) ** 1.5
    j = int(np.argmax(k[100:-100])) + 100
    return X[j], Y[j]


@pytest.mark.parametrize("decay,noise,nlam", [(1.0, 1e-4, 40),
                                              (1.5, 1e-3, 40),
                                              (2.0, 1e-2, 30),
                                              (0.7, 1e-3, 30),
                                              (1.0, 1e-2, 40)])
def test_corner_of_a_closed_form_lcurve(decay, noise, nlam):
    # discrete ill-posed problem: singular values k^-decay * e^-k/20,
    # coefficients of a smooth solution plus white noise
    k = np.arange(1, 201, dtype=float)
    s = k ** -decay * np.exp(-k / 20)
    rng = np.random.default_rng(3)
    beta = s * k ** -0.5 + noise * rng.standard_normal(k.size)
    lam = np.logspace(-6, 0, nlam)
    rho, eta = _tikhonov_curve(lam, s, beta)
    cx, cy = _true_corner(s, beta, -6, 0)
    d2 = (np.log10(rho) - cx) ** 2 + (np.log10(eta) - cy) ** 2
    want = int(np.argmin(d2))
    assert np.sort(d2)[1] > 1.5 * d2[want]        # an unambiguous case
    assert outer.lcurve_corner(lam, rho, eta) == want


def test_corner_of_two_straight_legs():
    # a vertical leg then a horizontal one in the log-log plane: the joint
    # is the corner
    lam = np.logspace(-3, 1, 21)
    j = 8
    X = np.where(np.arange(21) <= j, 0.0, 0.25 * (np.arange(21) - j))
    Y = np.where(np.arange(21) <= j, 0.25 * (j - np.arange(21)), 0.0)
    rho, eta = 10.0 ** X, 10.0 ** Y
    assert outer.lcurve_corner(lam, rho, eta) == j


def test_corner_scale_invariant():
    k = np.arange(1, 101, dtype=float)
    s = np.exp(-k / 12)
    beta = s * 0.9 ** k + 1e-3 * np.random.default_rng(5).standard_normal(100)
    lam = np.logspace(-5, 0, 25)
    rho, eta = _tikhonov_curve(lam, s, beta)
    c = outer.lcurve_corner(lam, rho, eta)
    assert outer.lcurve_corner(lam, 3.0 * rho, 0.01 * eta) == c
    assert outer.lcurve_corner(lam * 10.0, rho, eta) == c


# ---- trimming window and stopping rule -------------------------------------

def test_trim_window_examples():
    # ten lambdas from two below to seven above the previous choice,
    # shifted to the smallest or largest ten near the ends (0-based)
    assert outer.trim_window(5, 20) == (3, 12)
    assert outer.trim_window(0, 20) == (0, 9)
    assert outer.trim_window(1, 20) == (0, 9)
    assert outer.trim_window(2, 20) == (0, 9)
    assert outer.trim_window(3, 20) == (1, 10)
    assert outer.trim_window(12, 20) == (10, 19)
    assert outer.trim_window(19, 20) == (10, 19)
    for i in range(10):
        assert outer.trim_window(i, 10) == (0, 9)
    for m in (10, 17, 64):
        for i in range(m):
            lo, hi = outer.trim_window(i, m)
            assert hi - lo + 1 == 10 and 0 <= lo and hi <= m - 1
            assert lo <= i <= hi


def test_stop_rule():
    assert not outer.stop_rule([4])
    assert not outer.stop_rule([4, 4])
    assert outer.stop_rule([4, 4, 4])
    assert not outer.stop_rule([3, 4, 4])
    assert outer.stop_rule([2, 3, 4, 4, 4])
    assert not outer.stop_rule([4, 4, 5])
