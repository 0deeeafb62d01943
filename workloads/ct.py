"""Seeded tomography workloads: a parallel-beam projector by exact ray
lengths (Siddon's method) and an ellipse phantom.

Like the rest of this package these are inputs, shared unchanged by the
oracle and the GPU path: the projector is generated once here (FP32
values, as the tomography configuration stores them) and handed to both.

Geometry (unit pixels centred at the origin): pixel (i, j) of an N x N
image, index p = i + N j, covers x in [j - N/2, j + 1 - N/2] and
y in [i - N/2, i + 1 - N/2].  Angle k is theta_k = k pi / n_angles (full
angle), or k times a given step (limited angle, e.g. 0, 2, ..., 130 degrees
as in the paper's Section 4.5); bin b
is the offset s_b = b - (n_bins - 1) / 2; ray (k, b) is the line
x cos(theta) + y sin(theta) = s_b, row k * n_bins + b of A.  A[row, p] is
the length of the ray inside pixel p.  A ray lying exactly on a grid line
gives half its length to each of the two pixels it borders.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import (L_NEUMANN, add_noise, edge_weights, ellipse_phantom,
               lambda_grid, seed_for)


def _axis_ray(N: int, s: float):
    """Lengths of a ray parallel to an image axis at offset s (in the
    coordinate across the axis): (indices across the axis, weights)."""
    u = s + N / 2.0                       # position in pixel units from the edge
    if u < 0.0 or u > N:
        return [], []
    k = math.floor(u)
    if abs(u - round(u)) < 1e-9:          # exactly on a grid line: split
        k = int(round(u))
        out = [(k - 1, 0.5), (k, 0.5)]
        return [a for a, _ in out if 0 <= a < N], [w for a, w in out if 0 <= a < N]
    return [k], [1.0]


def parallel_beam(N: int, n_angles: int, n_bins: int,
                  angle_step: float | None = None):
    """CSR arrays (rowptr int64, col int32, val float32) of the parallel-beam
    projector, m = n_angles * n_bins rows, N * N columns, columns sorted
    within each row.  angle_step (radians): theta_k = k angle_step instead
    of k pi / n_angles."""
    rows, cols, vals = [], [], []
    s = np.arange(n_bins) - (n_bins - 1) / 2.0
    edges = np.arange(N + 1) - N / 2.0
    for k in range(n_angles):
        th = k * (math.pi / n_angles if angle_step is None else angle_step)
        c, sn = math.cos(th), math.sin(th)
        r0 = k * n_bins
        if abs(sn) < 1e-12 or abs(c) < 1e-12:
            # axis-aligned: theta = 0 gives vertical rays x = s (direction
            # +y), theta = pi/2 horizontal rays y = s
            vertical = abs(sn) < 1e-12
            for b in range(n_bins):
                across, w = _axis_ray(N, s[b] * (c if vertical else sn))
                for a, wa in zip(across, w):
                    line = np.arange(N)
                    if vertical:      # x fixed: column j = a, every row i
                        p = line + N * a
                    else:             # y fixed: row i = a, every column j
                        p = a + N * line
                    rows.append(np.full(N, r0 + b))
                    cols.append(p)
                    vals.append(np.full(N, wa))
            continue
        # points of ray b: (s_b c, s_b sn) + t (-sn, c)
        sx, sy = s * c, s * sn
        tx = (sx[:, None] - edges[None, :]) / sn          # x(t) = edge
        ty = (edges[None, :] - sy[:, None]) / c           # y(t) = edge
        # parameter interval inside the square
        ax = np.sort(np.stack([(sx - edges[0]) / sn, (sx - edges[-1]) / sn]), 0)
        ay = np.sort(np.stack([(edges[0] - sy) / c, (edges[-1] - sy) / c]), 0)
        tmin = np.maximum(ax[0], ay[0])
        tmax = np.minimum(ax[1], ay[1])
        t = np.concatenate([tx, ty], axis=1)
        t = np.clip(t, tmin[:, None], tmax[:, None])
        t = np.sort(np.concatenate([tmin[:, None], t, tmax[:, None]], 1), 1)
        seg = np.diff(t, axis=1)
        mid = 0.5 * (t[:, 1:] + t[:, :-1])
        xm = sx[:, None] - mid * sn
        ym = sy[:, None] + mid * c
        j = np.floor(xm + N / 2.0).astype(np.int64)
        i = np.floor(ym + N / 2.0).astype(np.int64)
        ok = (seg > 1e-12) & (i >= 0) & (i < N) & (j >= 0) & (j < N)
        ok &= (tmax > tmin)[:, None]
        rr = np.broadcast_to(np.arange(n_bins)[:, None] + r0, seg.shape)
        rows.append(rr[ok])
        cols.append((i + N * j)[ok])
        vals.append(seg[ok])
    row = np.concatenate(rows).astype(np.int64)
    col = np.concatenate(cols).astype(np.int64)
    val = np.concatenate(vals)
    m = n_angles * n_bins
    # canonical CSR: sorted columns, duplicates (a segment split across
    # neighbouring crossings at equal parameters) summed
    key = row * (N * N) + col
    order = np.argsort(key, kind="stable")
    key, val = key[order], val[order]
    uniq, start = np.unique(key, return_index=True)
    sums = np.add.reduceat(val, start)
    r = uniq // (N * N)
    cidx = (uniq % (N * N)).astype(np.int32)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cidx, sums.astype(np.float32)


@dataclass
class CtProblem:
    """One tomography workload: projector, data and sweep."""
    name: str
    N: int
    n_angles: int
    n_bins: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray              # float32
    levels: int
    x_true: np.ndarray
    b: np.ndarray                # m values
    lams: np.ndarray
    weights: list = field(default_factory=list)
    lbc: str = L_NEUMANN
    noise: float = 0.01

    @property
    def nv(self) -> int:
        return self.N

    @property
    def nh(self) -> int:
        return self.N

    @property
    def n(self) -> int:
        return self.N * self.N

    @property
    def m(self) -> int:
        return self.n_angles * self.n_bins

    def matrix(self):
        """The projector as a SciPy CSR matrix with FP64 copies of the FP32
        values (for the oracle)."""
        import scipy.sparse as sp
        return sp.csr_matrix((self.val.astype(np.float64), self.col,
                              self.rowptr), shape=(self.m, self.n))


def ct_problem(config: int, N: int, n_angles: int, n_bins: int | None,
               nellipses: int, noise: float, lams: np.ndarray, n_outer: int,
               levels: int, name: str = "",
               angle_step: float | None = None) -> CtProblem:
    nb = n_bins if n_bins is not None else math.ceil(N * math.sqrt(2.0))
    rp, ci, va = parallel_beam(N, n_angles, nb, angle_step)
    x = ellipse_phantom(N, nellipses, seed_for(config, 0, 1))
    import scipy.sparse as sp
    A = sp.csr_matrix((va.astype(np.float64), ci, rp), shape=(n_angles * nb, N * N))
    b = add_noise(A @ x, noise, seed_for(config, 0, 2))
    ws = [edge_weights(x, N, N, L_NEUMANN, ell, "fixed", seed_for(config))
          for ell in range(n_outer)]
    return CtProblem(name or f"ct{N}", N, n_angles, nb, rp, ci, va, levels, x,
                     b, np.asarray(lams, float), ws, L_NEUMANN, noise)


def config3() -> CtProblem:
    """256x256 parallel beam, 180 angles over [0, pi), 363 bins, 10-ellipse
    phantom, 1% noise, D = I and 0.01 on phantom edges, 32 lambdas in
    [1e-3, 1e2], 4 levels (coarsest 32x32)."""
    return ct_problem(3, 256, 180, 363, 10, 0.01, lambda_grid(-3, 2, 32), 2,
                      4, "ct256_parallel")


def small_ct(N: int = 32, n_angles: int = 24, levels: int = 3, nlam: int = 4,
             seed_cfg: int = 13) -> CtProblem:
    """A reduced tomography case with the same recipe (tests)."""
    return ct_problem(seed_cfg, N, n_angles, None, 4, 0.01,
                      lambda_grid(-3, 2, nlam), 2, levels, f"ct{N}_small")


def limited_angle_ct(N: int = 64, noise: float = 0.01, nlam: int = 30,
                     levels: int = 3, seed_cfg: int = 15) -> CtProblem:
    """Limited-angle parallel beam as in the paper's Section 4.5: 66 angles
    0, 2, ..., 130 degrees, ceil(N sqrt 2) bins, a seeded ellipse phantom
    (standing in for the paper's grains image), D = I and 0.01 on phantom
    edges, lambdas log-spaced in [1e-3, 1e2]."""
    return ct_problem(seed_cfg, N, 66, None, 6, noise,
                      lambda_grid(-3, 2, nlam), 2, levels,
                      f"ct{N}_limited_angle", angle_step=math.pi / 90)
