"""Pins of the CPU oracle against values fixed outside it.

Each test checks an oracle routine against something the oracle does not
compute itself: a library routine (scipy.ndimage, scipy.fft, numpy lstsq,
eigvalsh), a textbook value in tests/golden, a closed form, brute force on a
tiny input, or an invariant of the mathematics.
"""
import os

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.sparse as sp
from scipy.fft import dct
from scipy.special import eval_chebyt

import workloads as W
from oracle import direct
from oracle import operators as ops
from oracle.multigrid import (Hierarchy, VCycle, chebyshev, interpolation_1d,
                              SparseOp)
from oracle.pcg import DeblurOracle, pcg

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def _img(x, nv, nh):
    return x.reshape(nh, nv).T     # X[i, j]


# --------------------------------------------------------------- blur A
@pytest.mark.parametrize("bc,mode", [("periodic", "wrap"),
                                     ("reflective", "reflect"),
                                     ("zero", "constant")])
def test_blur_matches_scipy_convolve(bc, mode):
    nv, nh = 13, 10
    tv, th = W.gaussian_taps(3, 1.3), W.gaussian_taps(2, 0.9)
    x = RNG.standard_normal(nv * nh)
    A = ops.blur_matrix(tv, th, nv, nh, bc)
    X = _img(x, nv, nh)
    Y = ndi.convolve1d(X, tv, axis=0, mode=mode, cval=0.0)
    Y = ndi.convolve1d(Y, th, axis=1, mode=mode, cval=0.0)
    np.testing.assert_allclose(_img(A @ x, nv, nh), Y, rtol=0, atol=1e-14)


def test_blur_matches_generator_forward_model():
    nv, nh = 12, 9
    tv, th = W.gaussian_taps(2, 1.0), W.gaussian_taps(3, 1.5)
    x = RNG.standard_normal(nv * nh)
    for bc in ("periodic", "reflective", "zero"):
        A = ops.blur_matrix(tv, th, nv, nh, bc)
        np.testing.assert_allclose(A @ x, W.blur_data(x, nv, nh, tv, th, bc),
                                   atol=1e-14)


def test_asymmetric_taps_are_convolution():
    # (B x)_i = sum_k t_k x_{i-k}: a shifted delta moves the signal forward.
    taps = np.array([0.0, 0.0, 1.0])          # t_{+1} = 1
    B = ops.blur_matrix_1d(taps, 6, "zero").toarray()
    x = np.arange(1.0, 7.0)
    np.testing.assert_array_equal(B @ x, [0, 1, 2, 3, 4, 5])


@pytest.mark.parametrize("bc", ["periodic", "reflective"])
def test_blur_preserves_constants(bc):
    A = ops.blur_matrix(W.gaussian_taps(4, 2.0), W.gaussian_taps(3, 1.0),
                        16, 12, bc)
    np.testing.assert_allclose(A @ np.ones(16 * 12), 1.0, atol=1e-15)


def test_reflective_blur_diagonalized_by_dct():
    n = 24
    taps = W.gaussian_taps(5, 2.0)
    B = ops.blur_matrix_1d(taps, n, "reflective").toarray()
    C = dct(np.eye(n), type=2, norm="ortho", axis=0)     # orthonormal DCT-II
    T = C @ B @ C.T
    off = T - np.diag(np.diag(T))
    assert np.max(np.abs(off)) < 1e-14
    np.testing.assert_allclose(np.diag(T), direct.reflective_symbol(taps, n),
                               atol=1e-14)


def test_periodic_blur_eigenvalues_are_dft_of_taps():
    n = 16
    taps = W.gaussian_taps(3, 1.2)
    B = ops.blur_matrix_1d(taps, n, "periodic").toarray()
    ev = np.sort(np.linalg.eigvalsh(B))
    sym = np.zeros(n)
    sym[:4] = taps[3:]
    sym[-3:] = taps[:3]
    np.testing.assert_allclose(ev, np.sort(np.real(np.fft.fft(sym))),
                               atol=1e-14)


# --------------------------------------------------------------- gradient L
def _read_golden_rows(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([float(t) for t in line.replace("--", " ").split()])
    return rows


def test_gradient_hand_example():
    X = np.array([[1, 2, 4], [3, 5, 9], [6, 7, 8]], float)
    x = X.T.ravel()                               # column-major
    L = ops.gradient(3, 3, "neumann")
    g = L @ x
    gv, gh = _img(g[:9], 3, 3), _img(g[9:], 3, 3)
    want_v, want_h = _read_golden_rows("gradient_3x3.txt")
    np.testing.assert_array_equal(gv[:2, :].T.ravel(), want_v)
    np.testing.assert_array_equal(gh[:, :2].T.ravel(), want_h)
    assert np.all(gv[2, :] == 0) and np.all(gh[:, 2] == 0)   # padding rows


def test_padded_gradient_equals_paper_gradient():
    nv, nh = 5, 4
    Lv = sp.diags([-np.ones(nv - 1), np.ones(nv - 1)], [0, 1],
                  shape=(nv - 1, nv))
    Lh = sp.diags([-np.ones(nh - 1), np.ones(nh - 1)], [0, 1],
                  shape=(nh - 1, nh))
    Lpaper = sp.vstack([sp.kron(sp.identity(nh), Lv),
                        sp.kron(Lh, sp.identity(nv))]).toarray()
    L = ops.gradient(nv, nh, "neumann").toarray()
    keep = np.any(L != 0, axis=1)
    np.testing.assert_array_equal(L[keep], Lpaper)
    assert Lpaper.shape[0] == nh * (nv - 1) + (nh - 1) * nv


@pytest.mark.parametrize("lbc", ["neumann", "periodic"])
def test_gradient_kills_constants_and_laplacian(lbc):
    nv, nh = 6, 5
    L = ops.gradient(nv, nh, lbc)
    assert np.abs(L @ np.ones(nv * nh)).max() == 0
    lap = (L.T @ L).toarray()
    d = _img(np.diag(lap), nv, nh)
    if lbc == "periodic":
        assert np.all(d == 4)
    else:   # Neumann: 4 inside, 3 on edges, 2 at corners
        assert d[2, 2] == 4 and d[0, 2] == 3 and d[2, 0] == 3 and d[0, 0] == 2
        assert d[-1, -1] == 2


def test_normal_matrix_spd():
    nv, nh = 8, 6
    A = ops.blur_matrix(W.gaussian_taps(2, 1.0), W.gaussian_taps(2, 1.0),
                        nv, nh, "reflective")
    d = RNG.uniform(0.01, 1.0, 2 * nv * nh)
    K = ops.normal_matrix(A, ops.regularizer(d, nv, nh, "neumann"), 1e-2)
    K = K.toarray()
    assert np.abs(K - K.T).max() < 1e-15
    assert np.linalg.eigvalsh(K).min() > 0


# --------------------------------------------------------------- direct solves
@pytest.mark.parametrize("bc,lbc", [("periodic", "periodic"),
                                    ("reflective", "neumann"),
                                    ("zero", "neumann")])
def test_dense_equals_stacked_least_squares(bc, lbc):
    nv, nh = 8, 8
    A = ops.blur_matrix(W.gaussian_taps(2, 1.2), W.gaussian_taps(2, 1.2),
                        nv, nh, bc)
    d = RNG.uniform(0.01, 1.0, 2 * nv * nh)
    M = ops.regularizer(d, nv, nh, lbc)
    b = RNG.standard_normal(nv * nh)
    for lam in (1e-2, 1.0):
        xd = direct.solve_dense(A, M, b, lam)
        xs = direct.solve_stacked(A, M, b, lam)
        assert np.linalg.norm(xd - xs) <= 1e-9 * np.linalg.norm(xs)


def test_fft_closed_form_equals_dense():
    nv, nh = 16, 12
    tv, th = W.gaussian_taps(3, 1.5), W.gaussian_taps(2, 1.0)
    A = ops.blur_matrix(tv, th, nv, nh, "periodic")
    M = ops.regularizer(np.ones(2 * nv * nh), nv, nh, "periodic")
    b = RNG.standard_normal(nv * nh)
    for lam in (1e-3, 1e-1, 1.0):
        xd = direct.solve_dense(A, M, b, lam)
        xf = direct.solve_fft(tv, th, nv, nh, b, lam)
        assert np.linalg.norm(xd - xf) <= 1e-9 * np.linalg.norm(xd)


def test_dct_closed_form_equals_dense():
    nv, nh = 16, 12
    tv, th = W.gaussian_taps(3, 1.5), W.gaussian_taps(2, 1.0)
    A = ops.blur_matrix(tv, th, nv, nh, "reflective")
    M = ops.regularizer(np.ones(2 * nv * nh), nv, nh, "neumann")
    b = RNG.standard_normal(nv * nh)
    for lam in (1e-3, 1e-1, 1.0):
        xd = direct.solve_dense(A, M, b, lam)
        xc = direct.solve_dct(tv, th, nv, nh, b, lam)
        assert np.linalg.norm(xd - xc) <= 1e-9 * np.linalg.norm(xd)


@pytest.mark.parametrize("bc,lbc", [("periodic", "periodic"),
                                    ("reflective", "neumann")])
def test_reference_solve_with_weights_equals_dense(bc, lbc):
    nv, nh = 16, 16
    tv = W.gaussian_taps(3, 1.5)
    d = RNG.uniform(0.01, 1.0, 2 * nv * nh)
    O = DeblurOracle(nv, nh, tv, tv, bc, lbc, d)
    b = RNG.standard_normal(nv * nh)
    for lam in (1e-3, 1.0):
        xr, rel = O.reference(b, lam)
        xd = direct.solve_stacked(O.A.explicit(), O.M, b, lam)
        assert rel < 1e-12
        assert np.linalg.norm(xr - xd) <= 1e-8 * np.linalg.norm(xd)


# --------------------------------------------------------------- multigrid
def test_interpolation_hand_example():
    Pn = interpolation_1d(8, periodic=False).toarray()
    want = np.zeros((8, 4))
    for I in range(4):
        want[2 * I, I] = 1
    want[1, 0:2] = 0.5
    want[3, 1:3] = 0.5
    want[5, 2:4] = 0.5
    want[7, 3] = 1.0
    np.testing.assert_array_equal(Pn, want)
    Pp = interpolation_1d(8, periodic=True).toarray()
    want[7, 3] = 0.5
    want[7, 0] = 0.5
    np.testing.assert_array_equal(Pp, want)


@pytest.mark.parametrize("periodic", [False, True])
def test_interpolation_preserves_constants(periodic):
    P = sp.kron(interpolation_1d(16, periodic), interpolation_1d(8, periodic))
    np.testing.assert_array_equal(P @ np.ones(8 * 4), np.ones(16 * 8))


def test_galerkin_laplacian_textbook_stencil():
    nv = nh = 16
    L = ops.gradient(nv, nh, "neumann")
    S = (L.T @ L).tocsr()
    P = sp.kron(interpolation_1d(nh, False), interpolation_1d(nv, False))
    Sc = (P.T @ S @ P).toarray()
    ncv = nv // 2
    I, J = 3, 4                                       # interior coarse node
    row = Sc[I + ncv * J].reshape(nh // 2, ncv).T     # [i, j]
    got = row[I - 1:I + 2, J - 1:J + 2]
    want = np.loadtxt(os.path.join(GOLD, "galerkin_laplacian_9pt.txt"))
    np.testing.assert_allclose(got, want, atol=1e-15)
    np.testing.assert_allclose(Sc @ np.ones(ncv * nh // 2), 0, atol=1e-13)


def _small_oracle(bc="reflective", lbc="neumann", nv=16, nh=16, levels=3,
                  seed=3):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.01, 1.0, 2 * nv * nh)
    tv = W.gaussian_taps(2, 1.0)
    th = W.gaussian_taps(3, 1.4)
    return DeblurOracle(nv, nh, tv, th, bc, lbc, d, levels)


@pytest.mark.parametrize("bc,lbc", [("reflective", "neumann"),
                                    ("periodic", "periodic")])
def test_one_sided_hierarchy_is_galerkin(bc, lbc):
    O = _small_oracle(bc, lbc)
    H = O.H
    A = O.A.explicit()
    lam = 0.3
    K = ops.normal_matrix(A, O.M, lam).toarray()
    for k in range(1, H.levels):
        K = H.P[k - 1].T.toarray() @ K @ H.P[k - 1].toarray()
        n = H.nv[k] * H.nh[k]
        Kk = np.column_stack([H.K(k, lam, e) for e in np.eye(n)])
        np.testing.assert_allclose(Kk, K, atol=1e-13 * np.abs(K).max())
        np.testing.assert_allclose(H.diag(k, lam), np.diag(K), rtol=1e-13)
    np.testing.assert_allclose(H.coarse_matrix(lam), K,
                               atol=1e-13 * np.abs(K).max())


def test_gershgorin_bounds_spectrum():
    O = _small_oracle()
    H = O.H
    for lam in (1e-3, 1e-1, 3.0):
        for k in range(H.levels):
            n = H.nv[k] * H.nh[k]
            Kk = np.column_stack([H.K(k, lam, e) for e in np.eye(n)])
            dm = 1 / np.sqrt(H.diag(k, lam))
            mu = np.linalg.eigvalsh(dm[:, None] * Kk * dm[None, :]).max()
            g = H.gershgorin(k, lam)
            assert mu <= g * (1 + 1e-12)
            assert g <= 2.5 * mu          # not a vacuous bound


def test_gershgorin_tight_for_periodic_blur():
    # Nonnegative circulant: the constant vector attains the row sum.
    nv = nh = 16
    tv = W.gaussian_taps(3, 1.5)
    O = DeblurOracle(nv, nh, tv, tv, "periodic", "periodic",
                     np.ones(2 * nv * nh), 2)
    g = O.H.gershgorin(0, 0.0)
    diag = (tv @ tv) ** 2
    assert abs(g - 1.0 / diag) < 1e-10 * g


def test_chebyshev_polynomial():
    # Error propagation of `steps` Chebyshev steps on a diagonal operator
    # equals T_s((theta - mu)/delta) / T_s(theta/delta) at each eigenvalue.
    mu = np.linspace(0.05, 2.0, 40)
    K = lambda v: mu * v
    a, b = 0.4, 2.0
    theta, delta = (a + b) / 2, (b - a) / 2
    for steps in (1, 2, 3, 4):
        x0 = np.ones_like(mu)                       # error e0 = x0 - 0
        x = chebyshev(K, np.ones_like(mu), np.zeros_like(mu), x0, a, b, steps)
        want = eval_chebyt(steps, (theta - mu) / delta) / \
            eval_chebyt(steps, theta / delta)
        np.testing.assert_allclose(x, want, atol=1e-14)


def test_three_term_chebyshev_form_has_the_same_polynomial():
    # The tiled smoothing kernel runs the recurrence in three-term form,
    # x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 D^-1 (b - K x_k), with the
    # two-term coefficients c1 = rho_k rho_{k-1}, c2 = 2 rho_k / delta and
    # the first step x_1 = x_0 + D^-1 r_0 / theta.  Its error propagation
    # must be the same Chebyshev ratio T_s((theta - mu)/delta) / T_s(theta/delta).
    mu = np.linspace(0.05, 2.0, 40)
    a, b = 0.4, 2.0
    theta, delta = (a + b) / 2, (b - a) / 2
    sigma = theta / delta
    for steps in (1, 2, 3, 4, 6):
        x_prev = np.ones_like(mu)                  # x_0: error e0 = 1
        x = x_prev + (-mu * x_prev) / theta        # b = 0, D = I
        rho_old = 1.0 / sigma
        for _ in range(1, steps):
            rho = 1.0 / (2.0 * sigma - rho_old)
            c1, c2 = rho * rho_old, 2.0 * rho / delta
            x, x_prev = x + c1 * (x - x_prev) + c2 * (-mu * x), x
            rho_old = rho
        want = eval_chebyt(steps, (theta - mu) / delta) / \
            eval_chebyt(steps, theta / delta)
        np.testing.assert_allclose(x, want, atol=1e-14)


def test_coarse_correction_is_projection():
    O = _small_oracle(levels=2)
    H = O.H
    lam = 0.05
    n = H.nv[0] * H.nh[0]
    K = np.column_stack([H.K(0, lam, e) for e in np.eye(n)])
    P = H.P[0].toarray()
    Kc = H.coarse_matrix(lam)
    C = np.eye(n) - P @ np.linalg.solve(Kc, P.T @ K)
    np.testing.assert_allclose(C @ C, C, atol=1e-10)


@pytest.mark.parametrize("bc,lbc", [("reflective", "neumann"),
                                    ("periodic", "periodic")])
def test_vcycle_symmetric_positive_definite(bc, lbc):
    O = _small_oracle(bc, lbc)
    n = O.nv * O.nh
    for lam in (1e-3, 0.1, 2.0):
        V = O.vcycle(lam)
        Mm = np.column_stack([V(e) for e in np.eye(n)])
        assert np.abs(Mm - Mm.T).max() < 1e-10 * np.abs(Mm).max()
        assert np.linalg.eigvalsh(0.5 * (Mm + Mm.T)).min() > 0


def test_single_level_vcycle_is_exact_inverse():
    O = _small_oracle(levels=1, nv=8, nh=8)
    lam = 0.2
    V = O.vcycle(lam)
    f = RNG.standard_normal(64)
    K = ops.normal_matrix(O.A.explicit(), O.M, lam).toarray()
    np.testing.assert_allclose(K @ V(f), f, atol=1e-12)
    x, it, _, _ = O.mg_pcg(O.A.rmatvec(f), lam, tol=1e-12)
    assert it == 1


# --------------------------------------------------------------- PCG
def test_cg_finite_termination():
    Q, _ = np.linalg.qr(RNG.standard_normal((30, 30)))
    ev = np.repeat([1.0, 3.0, 10.0], 10)
    K = (Q * ev) @ Q.T
    f = RNG.standard_normal(30)
    x, it, nr, _ = pcg(lambda v: K @ v, f, tol=1e-12)
    assert it <= 3
    np.testing.assert_allclose(x, np.linalg.solve(K, f), atol=1e-10)


def test_cg_energy_error_monotone():
    n = 40
    Q, _ = np.linalg.qr(RNG.standard_normal((n, n)))
    K = (Q * np.geomspace(1e-2, 1, n)) @ Q.T
    f = RNG.standard_normal(n)
    xs = np.linalg.solve(K, f)
    errs = []
    for m in range(1, 25):
        x, _, _, _ = pcg(lambda v: K @ v, f, tol=0.0, maxit=m)
        e = x - xs
        errs.append(e @ K @ e)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))


def test_flexible_cg_equals_standard_cg_for_fixed_preconditioner():
    # With a fixed SPD preconditioner z_new . r_old = 0 in exact arithmetic,
    # so the Polak-Ribiere beta equals the Fletcher-Reeves one and the
    # iterates coincide (up to rounding).
    # Moderate conditioning and few steps, before rounding-driven loss of
    # orthogonality separates the two recurrences.
    n = 60
    Q, _ = np.linalg.qr(RNG.standard_normal((n, n)))
    K = (Q * np.geomspace(1e-1, 1, n)) @ Q.T
    G = RNG.standard_normal((n, n))
    Minv = G @ G.T + n * np.eye(n)
    f = RNG.standard_normal(n)
    for m in (3, 6, 10):
        xs, _, _, _ = pcg(lambda v: K @ v, f, lambda r: Minv @ r, tol=0.0,
                          maxit=m)
        xf, _, _, _ = pcg(lambda v: K @ v, f, lambda r: Minv @ r, tol=0.0,
                          maxit=m, flexible=True)
        assert np.linalg.norm(xf - xs) <= 1e-9 * np.linalg.norm(xs)


def test_flexible_cg_with_varying_preconditioner_reaches_solution():
    # A V-cycle evaluated in single precision is a slightly different map at
    # every application; flexible CG still reaches the FP64 solution, and its
    # iteration count stays close to that of the exact V-cycle.
    O = _small_oracle("reflective", "neumann", nv=32, nh=32, levels=3)
    b = RNG.standard_normal(32 * 32)
    lam = 1e-2
    V = O.vcycle(lam)
    V32 = lambda r: V(r.astype(np.float32).astype(np.float64)).astype(
        np.float32).astype(np.float64)
    K = O.K(lam)
    f = O.rhs(b)
    xd = direct.solve_stacked(O.A.explicit(), O.M, b, lam)
    x64, it64, _, _ = pcg(K, f, V, tol=1e-12)
    x32, it32, _, _ = pcg(K, f, V32, tol=1e-12, flexible=True)
    assert np.linalg.norm(x32 - xd) <= 1e-8 * np.linalg.norm(xd)
    assert it32 <= 1.1 * it64


@pytest.mark.parametrize("bc,lbc", [("reflective", "neumann"),
                                    ("periodic", "periodic")])
def test_mg_pcg_reaches_dense_solution(bc, lbc):
    O = _small_oracle(bc, lbc, nv=32, nh=32, levels=3)
    b = RNG.standard_normal(32 * 32)
    for lam in (1e-3, 0.1, 1.0):
        x, it, nr, _ = O.mg_pcg(b, lam, tol=1e-13)
        xd = direct.solve_stacked(O.A.explicit(), O.M, b, lam)
        assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)


def test_lcurve_monotone():
    P = W.small_deblur(32, 32, 3, 1.5, "reflective", "neumann", 3, nlam=8)
    O = DeblurOracle(P.nv, P.nh, P.taps_v, P.taps_h, P.bc, P.lbc,
                     P.weights[1], 3)
    pairs = [O.pair(O.reference(P.b, lam)[0], P.b) for lam in P.lams]
    rho = [p[0] for p in pairs]
    eta = [p[1] for p in pairs]
    assert all(b >= a * (1 - 1e-9) for a, b in zip(rho, rho[1:]))
    assert all(b <= a * (1 + 1e-9) for a, b in zip(eta, eta[1:]))


def test_sparse_operator_hierarchy_matches_kron():
    # The general (tomography) hierarchy path reproduces the Kronecker one.
    O = _small_oracle(levels=3)
    Hs = Hierarchy(SparseOp(O.A.explicit()), O.M, O.nv, O.nh, 3, False)
    Hk = O.H
    v = RNG.standard_normal(Hk.nv[2] * Hk.nh[2])
    np.testing.assert_allclose(Hs.K(2, 0.1, v), Hk.K(2, 0.1, v), atol=1e-13)
    np.testing.assert_allclose(Hs.diagA[1], Hk.diagA[1], rtol=1e-13)


def test_vcycle_contracts_laplacian_dominated_error():
    # With the regularization term dominant (large lambda, D = I), the
    # stationary iteration x <- x + V(f - K x) is a textbook multigrid
    # solver for a diffusion problem and must contract the error strongly.
    nv = nh = 32
    tv = W.gaussian_taps(2, 1.0)
    O = DeblurOracle(nv, nh, tv, tv, "reflective", "neumann",
                     np.ones(2 * nv * nh), 4)
    lam = 100.0
    V, K = O.vcycle(lam), O.K(lam)
    xs = RNG.standard_normal(nv * nh)
    f = K(xs)
    x = np.zeros_like(f)
    e0 = np.linalg.norm(xs)
    for _ in range(5):
        x = x + V(f - K(x))
    rate = (np.linalg.norm(xs - x) / e0) ** (1 / 5)
    assert rate < 0.15
