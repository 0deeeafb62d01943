"""Oracle for the outer reweighting loop of the paper's Algorithm 2.

Test infrastructure: only the tests, the smoke entry point and the CPU
baseline of the benchmark use this module; the library never does.

  * weight_update -- eq. (g) and the update D(l) = diag(d(l)) D(l-1)
    (Section 2): g = |D L x| / ||D L x||_inf elementwise, d = 1 - g^q;
  * lcurve_corner -- the L-curve of Section 1 (log10 of the residual norm
    against log10 of the weighted seminorm, parametrised by lambda) and the
    discrete lambda closest to the point of largest positive curvature of
    an interpolant through the points (the Hansen-O'Leary criterion the
    paper uses);
  * trim_window -- the pruned range of Section 3.4 and Algorithm 2: ten
    lambdas from two below to seven above the previous choice, shifted to
    the ends of the grid when near them;
  * stop_rule -- the stopping heuristic of Section 3.5: the same lambda
    chosen at three consecutive outer iterations;
  * regularize -- Algorithm 2 put together from the four, with every
    solve done by the oracle's reference solver.

Readings where the paper is silent:
  * ||D L x||_inf = 0 gives g = 0, so d = 1 and D is unchanged (the paper
    notes that case leaves D as it was);
  * the interpolant is a pair of natural cubic splines of log10 rho and
    log10 eta over log10 lambda through every point; its curvature is
    sampled at 64 points per interval (both ends included once) and the
    chosen lambda is the data point nearest, in the log-log plane, to the
    sample of largest curvature;
  * lambdas are given strictly increasing (Algorithm 2 indexes them from
    the smallest up); indices here are 0-based.
"""
import numpy as np
from scipy.interpolate import CubicSpline

from . import operators as ops

CORNER_SAMPLES = 64


def weight_update(d_prev, x, nv, nh, lbc, q):
    """eq. (g): returns (D(l) as 2n weights, ||D(l-1) L x||_inf)."""
    d_prev = np.asarray(d_prev, dtype=np.float64)
    w = np.abs(ops.regularizer(d_prev, nv, nh, lbc) @ np.asarray(x, float))
    top = float(w.max())
    g = w / top if top > 0.0 else np.zeros_like(w)
    return (1.0 - g ** q) * d_prev, top


def lcurve_curvature(lam, rho, eta, samples=CORNER_SAMPLES):
    """Samples (t, X, Y, kappa) of the interpolated L-curve, t = log10 lam."""
    t = np.log10(np.asarray(lam, float))
    X = CubicSpline(t, np.log10(np.asarray(rho, float)), bc_type="natural")
    Y = CubicSpline(t, np.log10(np.asarray(eta, float)), bc_type="natural")
    tt = [t[i] + (t[i + 1] - t[i]) * np.arange(samples) / samples
          for i in range(len(t) - 1)]
    tt = np.concatenate(tt + [t[-1:]])
    x1, x2 = X(tt, 1), X(tt, 2)
    y1, y2 = Y(tt, 1), Y(tt, 2)
    kappa = (x1 * y2 - y1 * x2) / (x1 * x1 + y1 * y1) ** 1.5
    return tt, X(tt), Y(tt), kappa


def lcurve_corner(lam, rho, eta, samples=CORNER_SAMPLES):
    """Index of the lambda closest to the L-curve's corner (Section 1)."""
    lam = np.asarray(lam, float)
    assert len(lam) >= 3 and np.all(np.diff(lam) > 0)
    _, xs, ys, kappa = lcurve_curvature(lam, rho, eta, samples)
    k = int(np.argmax(kappa))
    px = np.log10(np.asarray(rho, float))
    py = np.log10(np.asarray(eta, float))
    return int(np.argmin((px - xs[k]) ** 2 + (py - ys[k]) ** 2))


def trim_window(i_prev, m, size=10):
    """Inclusive index range [lo, hi] of the pruned sweep (Section 3.4)."""
    lo = max(min(i_prev - 2, m - size), 0)
    hi = min(max(i_prev + size - 3, size - 1), m - 1)
    return lo, hi


def stop_rule(chosen):
    """Section 3.5: stop once the last three choices are equal."""
    return len(chosen) >= 3 and chosen[-1] == chosen[-2] == chosen[-3]


def regularize(make_oracle, b, lam, q, maxouter, nv, nh, lbc):
    """Algorithm 2 with exact solves.  make_oracle(d) returns the oracle
    object (DeblurOracle or CtOracle) for weights d.  Returns the chosen
    solution, the chosen indices per outer iteration, the weights of the
    last solve (None for D = I) and whether the stopping rule fired."""
    lam = np.asarray(lam, float)
    m = len(lam)
    d = None
    chosen = []
    x_star = None
    for ell in range(maxouter):
        lo, hi = (0, m - 1) if ell == 0 else trim_window(chosen[-1], m)
        O = make_oracle(d)
        xs = [O.reference(b, lam[i])[0] for i in range(lo, hi + 1)]
        pairs = np.array([O.pair(x, b) for x in xs])
        c = lcurve_corner(lam[lo:hi + 1], pairs[:, 0], pairs[:, 1])
        chosen.append(lo + c)
        x_star = xs[c]
        if stop_rule(chosen):
            return x_star, chosen, d, True
        if ell + 1 < maxouter:
            d_prev = np.ones(2 * nv * nh) if d is None else d
            d, _ = weight_update(d_prev, x_star, nv, nh, lbc, q)
    return x_star, chosen, d, False
