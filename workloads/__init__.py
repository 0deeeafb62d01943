"""Seeded synthetic inputs for the regularized least-squares sweep.

This module produces the *inputs* of the method -- phantoms, point-spread
function taps, measured data, edge weights for the diagonal weighting matrix,
regularization-parameter grids and (for tomography) the projector matrix.  It
holds none of the solver's arithmetic: both the CPU oracle and the GPU path
consume what it returns and neither shares code with the other through it.

The paper's test images (Shepp-Logan via PRtomo, "grains" via PRset) and its
noise routine (PRnoise) are not available here; seeded stand-ins with the same
character (piecewise-constant images, white Gaussian noise scaled to a relative
level) replace them.  Measured data are simulated as ``b = A x_true + eta``
(the data model of the paper's Section 2, eq. (exact)) by a direct padded
convolution written here for data synthesis only.

Seeds follow ``seed = 1000*config + 10*outer_index + item``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Boundary condition names shared by the generators and the consumers.
BC_PERIODIC = "periodic"
BC_REFLECTIVE = "reflective"   # half-sample symmetric: x[-1] = x[0]
BC_ZERO = "zero"

L_NEUMANN = "neumann"          # last forward difference in each direction is 0
L_PERIODIC = "periodic"        # wrap-around forward difference


def seed_for(config: int, outer: int = 0, item: int = 0) -> int:
    return 1000 * config + 10 * outer + item


def lambda_grid(lo_exp: float, hi_exp: float, count: int) -> np.ndarray:
    """Log-spaced regularization parameters, increasing (smallest first)."""
    return np.logspace(lo_exp, hi_exp, count)


def gaussian_taps(r: int, sigma: float) -> np.ndarray:
    """Samples exp(-j^2 / (2 sigma^2)), j = -r..r, normalized to sum 1.

    A 2D separable PSF built from two such vectors also sums to 1.
    """
    j = np.arange(-r, r + 1, dtype=np.float64)
    t = np.exp(-(j * j) / (2.0 * sigma * sigma))
    return t / t.sum()


def shapes_phantom(nv: int, nh: int, nshapes: int, seed: int) -> np.ndarray:
    """Piecewise-constant image: random rectangles and disks, values U[0,1].

    Painted in order onto a zero background.  Returned column-major as a
    flat vector of length nv*nh with index i + nv*j (i vertical).
    """
    rng = np.random.default_rng(seed)
    img = np.zeros((nh, nv))  # img[j, i] so that ravel() is i-fastest
    ii = np.arange(nv)[None, :]
    jj = np.arange(nh)[:, None]
    for s in range(nshapes):
        val = rng.uniform(0.0, 1.0)
        if rng.uniform() < 0.5:
            hi = int(rng.integers(max(2, nv // 10), max(3, nv // 3)))
            wj = int(rng.integers(max(2, nh // 10), max(3, nh // 3)))
            i0 = int(rng.integers(0, nv - hi))
            j0 = int(rng.integers(0, nh - wj))
            img[j0:j0 + wj, i0:i0 + hi] = val
        else:
            rad = rng.uniform(0.05, 0.18) * min(nv, nh)
            ci = rng.uniform(rad, nv - rad)
            cj = rng.uniform(rad, nh - rad)
            mask = (ii - ci) ** 2 + (jj - cj) ** 2 <= rad * rad
            img[mask] = val
    return img.ravel().copy()


def ellipse_phantom(n: int, nellipses: int, seed: int) -> np.ndarray:
    """Ellipses inside the inscribed circle of an n x n image, values U[0,1]."""
    rng = np.random.default_rng(seed)
    img = np.zeros((n, n))
    c = (n - 1) / 2.0
    yy, xx = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    for e in range(nellipses):
        val = rng.uniform(0.0, 1.0)
        a = rng.uniform(0.08, 0.4) * n / 2
        b = rng.uniform(0.08, 0.4) * n / 2
        ang = rng.uniform(0, math.pi)
        rmax = n / 2 - max(a, b) - 1
        rr = rng.uniform(0, max(rmax, 0.0))
        th = rng.uniform(0, 2 * math.pi)
        x0, y0 = rr * math.cos(th), rr * math.sin(th)
        ca, sa = math.cos(ang), math.sin(ang)
        u = (xx - x0) * ca + (yy - y0) * sa
        v = -(xx - x0) * sa + (yy - y0) * ca
        img[(u / a) ** 2 + (v / b) ** 2 <= 1.0] = val
    return img.ravel().copy()


def _pad_index(idx: np.ndarray, n: int, bc: str):
    if bc == BC_PERIODIC:
        return np.mod(idx, n), np.ones(idx.shape, bool)
    if bc == BC_REFLECTIVE:
        m = np.mod(idx, 2 * n)
        return np.where(m < n, m, 2 * n - 1 - m), np.ones(idx.shape, bool)
    ok = (idx >= 0) & (idx < n)
    return np.clip(idx, 0, n - 1), ok


def blur_data(x: np.ndarray, nv: int, nh: int, taps_v: np.ndarray,
              taps_h: np.ndarray, bc: str) -> np.ndarray:
    """Simulate blurred data: 2D separable convolution of the image with the
    PSF t_v t_h^T under the given boundary extension (data synthesis only)."""
    img = x.reshape(nh, nv)                      # img[j, i]
    rv, rh = (len(taps_v) - 1) // 2, (len(taps_h) - 1) // 2
    out = np.zeros_like(img)
    iv = np.arange(nv)
    for k in range(-rv, rv + 1):
        src, ok = _pad_index(iv - k, nv, bc)
        out += taps_v[k + rv] * np.where(ok[None, :], img[:, src], 0.0)
    img2 = out
    out = np.zeros_like(img2)
    jh = np.arange(nh)
    for k in range(-rh, rh + 1):
        src, ok = _pad_index(jh - k, nh, bc)
        out += taps_h[k + rh] * np.where(ok[:, None], img2[src, :], 0.0)
    return out.ravel().copy()


def add_noise(b_true: np.ndarray, level: float, seed: int) -> np.ndarray:
    """b = b_true + level * ||b_true|| * e / ||e||, e ~ N(0, I)."""
    e = np.random.default_rng(seed).standard_normal(b_true.shape)
    return b_true + level * np.linalg.norm(b_true) * e / np.linalg.norm(e)


def phantom_edges(x: np.ndarray, nv: int, nh: int, lbc: str):
    """Boolean masks (vertical plane, horizontal plane) of gradient entries
    where the phantom changes between adjacent pixels."""
    img = x.reshape(nh, nv)
    if lbc == L_PERIODIC:
        dv = np.roll(img, -1, axis=1) - img
        dh = np.roll(img, -1, axis=0) - img
    else:
        dv = np.zeros_like(img)
        dh = np.zeros_like(img)
        dv[:, :-1] = img[:, 1:] - img[:, :-1]
        dh[:-1, :] = img[1:, :] - img[:-1, :]
    return (dv != 0).ravel(), (dh != 0).ravel()


def edge_weights(x: np.ndarray, nv: int, nh: int, lbc: str, outer: int,
                 scheme: str, seed_base: int, floor: float = 0.01) -> np.ndarray:
    """Diagonal of D^(outer) over the two gradient planes (vertical, then
    horizontal), length 2*nv*nh.

    outer == 0 gives D = I (the paper's starting weight).  For outer >= 1:
      scheme "fixed":   0.01 on phantom edges, 1 elsewhere;
      scheme "uniform": D^(l) = diag(u^(l)) D^(l-1) with u ~ U[0.01, 1] on
                        phantom edges and 1 elsewhere, clipped below at 0.01
                        (mirrors the multiplicative update D^(l) =
                        diag(d^(l)) D^(l-1) of the paper's Section 2).
    """
    n = nv * nh
    d = np.ones(2 * n)
    if outer == 0:
        return d
    ev, eh = phantom_edges(x, nv, nh, lbc)
    edges = np.concatenate([ev, eh])
    if scheme == "fixed":
        d[edges] = floor
        return d
    for ell in range(1, outer + 1):
        rng = np.random.default_rng(seed_base + 10 * ell + 7)
        u = np.ones(2 * n)
        u[edges] = rng.uniform(floor, 1.0, size=int(edges.sum()))
        d = np.maximum(d * u, floor)
    return d


@dataclass
class DeblurProblem:
    """One deblurring workload: operator description, data and sweep."""
    name: str
    nv: int
    nh: int
    taps_v: np.ndarray
    taps_h: np.ndarray
    bc: str
    lbc: str
    levels: int
    x_true: np.ndarray
    b: np.ndarray
    lams: np.ndarray
    weights: list = field(default_factory=list)   # one 2n vector per outer l
    tol: float = 1e-8
    noise: float = 0.01

    @property
    def n(self) -> int:
        return self.nv * self.nh


def deblur_problem(config: int, nv: int, nh: int, r: int, sigma: float,
                   bc: str, lbc: str, nshapes: int, noise: float,
                   lams: np.ndarray, n_outer: int, scheme: str, levels: int,
                   tol: float, name: str = "") -> DeblurProblem:
    x = shapes_phantom(nv, nh, nshapes, seed_for(config, 0, 1))
    tv = gaussian_taps(r, sigma)
    th = gaussian_taps(r, sigma)
    b_true = blur_data(x, nv, nh, tv, th, bc)
    b = add_noise(b_true, noise, seed_for(config, 0, 2))
    ws = [edge_weights(x, nv, nh, lbc, ell, scheme, seed_for(config))
          for ell in range(n_outer)]
    return DeblurProblem(name or f"deblur{nv}x{nh}", nv, nh, tv, th, bc, lbc,
                         levels, x, b, np.asarray(lams, float), ws, tol, noise)


def config1() -> DeblurProblem:
    """64x64, 9x9 Gaussian PSF sigma=2, periodic blur and gradient, 6 shapes,
    1% noise, D = I then 0.01 on edges, 8 lambdas in [1e-4, 1], tol 1e-8,
    3 multigrid levels (coarsest 16x16), FP64."""
    return deblur_problem(1, 64, 64, 4, 2.0, BC_PERIODIC, L_PERIODIC, 6, 0.01,
                          lambda_grid(-4, 0, 8), 2, "fixed", 3, 1e-8,
                          "deblur64_periodic_fp64")


def config2() -> DeblurProblem:
    """512x512, 15x15 Gaussian PSF sigma=3, reflective blur, Neumann
    gradient, 16 shapes, 1% noise, 3 outer weightings (D = I, then seeded
    U[0.01,1] edge weights), 20 lambdas in [1e-5, 1], 6 levels, tol 1e-8."""
    return deblur_problem(2, 512, 512, 7, 3.0, BC_REFLECTIVE, L_NEUMANN, 16,
                          0.01, lambda_grid(-5, 0, 20), 3, "uniform", 6, 1e-8,
                          "deblur512_reflective_fp64")


def config4() -> DeblurProblem:
    """2048x2048, 21x21 Gaussian PSF sigma=4, reflective blur, Neumann
    gradient, 16 shapes, 0.5% noise, 64 lambdas in [1e-4, 1], D = I and one
    edge-weighted outer step, 8 levels (coarsest 16x16)."""
    return deblur_problem(4, 2048, 2048, 10, 4.0, BC_REFLECTIVE, L_NEUMANN, 16,
                          0.005, lambda_grid(-4, 0, 64), 2, "fixed", 8, 1e-8,
                          "deblur2048_reflective_mixed")


def paper_deblur(n: int = 64, noise: float = 0.01, nlam: int = 30,
                 seed_cfg: int = 6) -> DeblurProblem:
    """The deblurring problem of the paper's Section 4.6 on an n x n grid:
    zero-boundary (Toeplitz) Kronecker blur with anisotropic truncated
    Gaussians, radius 6 and sigma 1.25 n / 64 along the contiguous axis,
    radius 7 and sigma 1.5 n / 64 across it, each normalized so that the
    symmetric kernel sums to one; Neumann gradient; a seeded shapes phantom
    (standing in for the paper's grains image); D = I, then 0.01 on phantom
    edges; lambdas log-spaced in [1e-3, 1e2]; levels down to a 16 x 16
    coarsest grid."""
    x = shapes_phantom(n, n, 12, seed_for(seed_cfg, 0, 1))
    tv = gaussian_taps(6, 1.25 * n / 64)
    th = gaussian_taps(7, 1.5 * n / 64)
    b = add_noise(blur_data(x, n, n, tv, th, BC_ZERO), noise,
                  seed_for(seed_cfg, 0, 2))
    ws = [edge_weights(x, n, n, L_NEUMANN, ell, "fixed", seed_for(seed_cfg))
          for ell in range(2)]
    levels = int(np.log2(n // 16)) + 1
    return DeblurProblem(f"paper_deblur{n}", n, n, tv, th, BC_ZERO, L_NEUMANN,
                         levels, x, b, lambda_grid(-3, 2, nlam), ws, 1e-8,
                         noise)


def small_deblur(nv: int, nh: int, r: int, sigma: float, bc: str, lbc: str,
                 levels: int, nlam: int = 4, seed_cfg: int = 9,
                 outer: int = 1, scheme: str = "uniform",
                 noise: float = 0.01) -> DeblurProblem:
    """A reduced-size deblurring case with the same recipe (tests)."""
    return deblur_problem(seed_cfg, nv, nh, r, sigma, bc, lbc,
                          max(3, min(16, nv * nh // 256)), noise,
                          lambda_grid(-4, 0, nlam), outer + 1, scheme, levels,
                          1e-8, f"small{nv}x{nh}_{bc}")
