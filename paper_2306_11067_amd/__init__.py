"""Batched multigrid-preconditioned lambda-sweep solver for regularized least
squares on MI355X.

Thin Python binding over librls.so (include/rls.h): it checks tensor
dtypes/devices and passes raw pointers and torch's current HIP stream.  No
arithmetic of the solver happens here and there is no CPU fallback: if the
library is not built, every call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

__all__ = ["Problem", "RLSError", "BC", "LBC"]

BC = {"periodic": L.RLS_BC_PERIODIC, "reflective": L.RLS_BC_REFLECTIVE,
      "zero": L.RLS_BC_ZERO}
LBC = {"neumann": L.RLS_L_NEUMANN, "periodic": L.RLS_L_PERIODIC}
PREC = {"fp64": L.RLS_PREC_FP64, "mixed_fp32": L.RLS_PREC_MIXED_FP32,
        "mixed_bf16": L.RLS_PREC_MIXED_BF16}


class RLSError(RuntimeError):
    """A failed library call: `status` is the RLS_E_* code, the message the
    library's own description of the failure."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int):
    if status != L.RLS_OK:
        raise RLSError(status, L.load().rls_last_error().decode())


def _dptr(t, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dbl(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """One regularized least-squares problem (A, L, grid) on the GPU."""

    def __init__(self, nv, nh, taps_v, taps_h, bc="reflective", lbc="neumann",
                 levels=3, nu=2, cheb_ratio=4.0, weights=None, nu_coarse=0,
                 cheb_ratio_coarse=0.0, precision="fp64"):
        self._lib = L.load()
        self.nv, self.nh, self.levels = int(nv), int(nh), int(levels)
        self.n = self.nv * self.nh
        tv, ptv = _dbl(taps_v)
        th, pth = _dbl(taps_h)
        op = L.OpDesc()
        op.kind = L.RLS_OP_BLUR_SEPARABLE
        op.bc = BC[bc]
        op.r_v = (len(tv) - 1) // 2
        op.r_h = (len(th) - 1) // 2
        op.taps_v, op.taps_h = ptv, pth
        g = L.GridDesc(self.nv, self.nh, LBC[lbc], self.levels, int(nu),
                       float(cheb_ratio), PREC[precision], int(nu_coarse),
                       float(cheb_ratio_coarse))
        h = C.c_void_p()
        d = None if weights is None else _dptr(weights, "weights", 2 * self.n)
        _check(self._lib.rls_setup(C.byref(h), C.byref(op), C.byref(g), d,
                                   _stream()))
        self._h = h
        self.m = self.n          # data values (A is square for the blur)

    def close(self):
        """Free the problem's device memory (idempotent)."""
        if getattr(self, "_h", None):
            self._lib.rls_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ main ABI
    def set_weights(self, weights=None):
        """Install the weights D of a new outer iteration (2n FP64 values on
        the device, vertical-difference plane first; None for D = I) and
        rebuild the coarse stencils of L^T D^2 L (paper Section 3.2)."""
        d = None if weights is None else _dptr(weights, "weights", 2 * self.n)
        _check(self._lib.rls_set_weights(self._h, d, _stream()))

    def solve_sweep(self, b, lams, tol, x0=None, x=None, maxit=100000,
                    tol_mode="relative", poll_every=32, graph=True):
        """Solve (A^T A + lambda^2 L^T D^2 L) x = A^T b for every lambda at
        once (batched PCG with the multigrid V-cycle).

        b: device FP64 data (m values); lams: the lambdas (> 0, any order);
        tol: residual target, relative to ||A^T b|| or absolute
        (tol_mode); x0: optional device warm starts, len(lams) * n values;
        x: optional output buffer (may be x0).  poll_every: iterations
        between host convergence checks; graph: replay iteration chunks as
        HIP graphs (same results either way).

        Returns (x viewed as (len(lams), n), ||A x - b|| per lambda,
        ||D L x|| per lambda, per-lambda dicts with iters, flags, relres
        (recursive) and relres_true (recomputed in FP64))."""
        import torch
        lam, plam = _dbl(lams)
        nl = len(lam)
        if x is None:
            x = torch.empty(nl * self.n, dtype=torch.float64, device=b.device)
        opts = L.SweepOpts(int(maxit), L.RLS_TOL_ABSOLUTE if tol_mode ==
                           "absolute" else L.RLS_TOL_RELATIVE, int(poll_every),
                           1 if graph else 0)
        res = np.zeros(nl)
        sem = np.zeros(nl)
        info = (L.SolveInfo * nl)()
        _check(self._lib.rls_solve_sweep(
            self._h, _dptr(b, "b", self.m), plam, nl, float(tol),
            C.byref(opts), None if x0 is None else _dptr(x0, "x0", nl * self.n),
            _dptr(x, "x", nl * self.n),
            res.ctypes.data_as(C.POINTER(C.c_double)),
            sem.ctypes.data_as(C.POINTER(C.c_double)), info, _stream()))
        inf = [dict(iters=i.iters, flags=i.flags, relres=i.relres,
                    relres_true=i.relres_true) for i in info]
        return x.view(nl, self.n), res, sem, inf

    # ---------------------------------------------------- outer loop ABI
    def update_weights(self, x, q):
        """eq. (g) from the solution x (device, n values); returns
        ||D L x||_inf."""
        top = C.c_double()
        _check(self._lib.rls_update_weights(self._h, _dptr(x, "x", self.n),
                                            float(q), C.byref(top), _stream()))
        return top.value

    def weights(self):
        """The current weights D (2n FP64 values on the device)."""
        import torch
        out = torch.empty(2 * self.n, dtype=torch.float64, device="cuda")
        _check(self._lib.rls_get_weights(self._h, _dptr(out, "d"), _stream()))
        return out

    def regularize(self, b, lams, q, tol, maxouter=10, maxit=100000,
                   tol_mode="relative", poll_every=32, graph=True):
        """Algorithm 2; returns (x, chosen indices, info dict)."""
        import torch
        lam, plam = _dbl(lams)
        opts = L.SweepOpts(int(maxit), L.RLS_TOL_ABSOLUTE if tol_mode ==
                           "absolute" else L.RLS_TOL_RELATIVE, int(poll_every),
                           1 if graph else 0)
        chosen = (C.c_int * int(maxouter))()
        info = L.OuterInfo()
        x = torch.empty(self.n, dtype=torch.float64, device=b.device)
        _check(self._lib.rls_regularize(
            self._h, _dptr(b, "b", self.m), plam, len(lam), float(q),
            float(tol), C.byref(opts), int(maxouter), chosen, _dptr(x, "x"),
            C.byref(info), _stream()))
        return x, list(chosen)[:info.outer], dict(
            outer=info.outer, stopped=bool(info.stopped),
            chosen_index=info.chosen_index, iters=info.iters)

    # ------------------------------------------------------------ step ABI
    def level_shape(self, level):
        """(nv, nh) of a multigrid level (0 is the finest)."""
        a, b = C.c_int(), C.c_int()
        _check(self._lib.rls_level_shape(self._h, level, C.byref(a), C.byref(b)))
        return a.value, b.value

    def apply_normal(self, level, lams, v):
        """K_k(lambda) v on a level for each lambda (v: device, one vector
        of the level per lambda, concatenated)."""
        import torch
        lam, plam = _dbl(lams)
        nv, nh = self.level_shape(level)
        out = torch.empty(len(lam) * nv * nh, dtype=torch.float64,
                          device=v.device)
        _check(self._lib.rls_apply_normal(
            self._h, level, plam, len(lam), _dptr(v, "v", len(lam) * nv * nh),
            _dptr(out, "out"), _stream()))
        return out

    def vcycle(self, lams, r):
        """One V-cycle z = M^{-1} r per lambda (paper Algorithm 1), with the
        problem's smoothing settings and precision."""
        import torch
        lam, plam = _dbl(lams)
        z = torch.empty_like(r)
        _check(self._lib.rls_vcycle(self._h, plam, len(lam),
                                    _dptr(r, "r", len(lam) * self.n),
                                    _dptr(z, "z"), _stream()))
        return z

    def stencil(self, level):
        """The level's stencil planes of L^T D^2 L (5 x n_k, host copy)."""
        nv, nh = self.level_shape(level)
        out = np.zeros(5 * nv * nh)
        _check(self._lib.rls_get_stencil(
            self._h, level, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(5, nv * nh)

    def gram_band(self, level, direction):
        """The level's 1D Gram band of the blur in one direction (0: along
        the contiguous axis, 1: across it), host copy."""
        bw = C.c_int()
        _check(self._lib.rls_get_gram_band(self._h, level, direction,
                                           C.byref(bw), None))
        nv, nh = self.level_shape(level)
        n = nv if direction == 0 else nh
        out = np.zeros(n * (2 * bw.value + 1))
        _check(self._lib.rls_get_gram_band(
            self._h, level, direction, C.byref(bw),
            out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(n, 2 * bw.value + 1)

    def gershgorin(self, level, lams):
        """Gershgorin bound of diag(K_k)^-1 K_k per lambda (the top of the
        Chebyshev smoothing interval)."""
        lam, plam = _dbl(lams)
        rho = np.zeros(len(lam))
        _check(self._lib.rls_gershgorin(
            self._h, level, plam, len(lam),
            rho.ctypes.data_as(C.POINTER(C.c_double)), _stream()))
        return rho

    def kernel_timer(self, enable=True):
        """Time the FP64 finest-level smoothing launches (HIP events around
        each run of consecutive launches; graphs are off while it is on)."""
        _check(self._lib.rls_kernel_timer(self._h, 1 if enable else 0))

    def kernel_timer_read(self):
        """(launches, seconds, algorithmic bytes) since the timer was enabled."""
        n, sec, byt = C.c_longlong(), C.c_double(), C.c_double()
        _check(self._lib.rls_kernel_timer_read(self._h, C.byref(n),
                                               C.byref(sec), C.byref(byt)))
        return n.value, sec.value, byt.value

    def forward(self, x, nvec=1):
        """y = A x for nvec vectors on the device."""
        import torch
        y = torch.empty(nvec * self.m, dtype=torch.float64, device=x.device)
        _check(self._lib.rls_apply_forward(self._h, _dptr(x, "x", nvec * self.n),
                                           _dptr(y, "y"), nvec, _stream()))
        return y

    def adjoint(self, y, nvec=1):
        """x = A^T y for nvec vectors on the device."""
        import torch
        x = torch.empty(nvec * self.n, dtype=torch.float64, device=y.device)
        _check(self._lib.rls_apply_adjoint(self._h, _dptr(y, "y", nvec * self.m),
                                           _dptr(x, "x"), nvec, _stream()))
        return x


class TomographyProblem(Problem):
    """A lambda-sweep problem with a general sparse forward operator (CSR,
    FP32 values >= 0, columns sorted within rows; e.g. the parallel-beam
    projector of workloads.ct).  Runs with the FP32 V-cycle under flexible
    FP64 PCG; b has m values."""

    def __init__(self, rowptr, col, val, N, levels=4, nu=2, cheb_ratio=4.0,
                 weights=None, lbc="neumann", nu_coarse=0,
                 cheb_ratio_coarse=0.0):
        self._lib = L.load()
        self.nv = self.nh = int(N)
        self.levels = int(levels)
        self.n = self.nv * self.nh
        self._rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._ci = np.ascontiguousarray(col, dtype=np.int32)
        self._va = np.ascontiguousarray(val, dtype=np.float32)
        self.m = len(self._rp) - 1
        op = L.OpDesc()
        op.kind = L.RLS_OP_CSR
        op.m = self.m
        op.nnz = len(self._ci)
        op.rowptr = self._rp.ctypes.data_as(C.POINTER(C.c_int64))
        op.col = self._ci.ctypes.data_as(C.POINTER(C.c_int32))
        op.val = self._va.ctypes.data_as(C.POINTER(C.c_float))
        g = L.GridDesc(self.nv, self.nh, LBC[lbc], self.levels, int(nu),
                       float(cheb_ratio), L.RLS_PREC_MIXED_FP32, int(nu_coarse),
                       float(cheb_ratio_coarse))
        h = C.c_void_p()
        d = None if weights is None else _dptr(weights, "weights", 2 * self.n)
        _check(self._lib.rls_setup(C.byref(h), C.byref(op), C.byref(g), d,
                                   _stream()))
        self._h = h


def lcurve_corner(lams, rho, eta):
    """Index of the L-curve corner (host computation in the library)."""
    lam, plam = _dbl(lams)
    r, pr = _dbl(rho)
    e, pe = _dbl(eta)
    idx = C.c_int()
    _check(L.load().rls_lcurve_corner(plam, pr, pe, len(lam), C.byref(idx)))
    return idx.value


def trim_window(i_prev, m):
    """Inclusive (lo, hi) of the pruned lambda range."""
    lo, hi = C.c_int(), C.c_int()
    _check(L.load().rls_trim_window(int(i_prev), int(m), C.byref(lo),
                                    C.byref(hi)))
    return lo.value, hi.value


def solve_batch(entries):
    """Solve the lambda sweeps of several problems together (rls_solve_batch).

    entries: list of dicts with keys prob, b, lams, tol and optionally x0,
    maxit, tol_mode, poll_every, graph.  Returns a list of (x, resnorm,
    seminorm, info) in the order of `entries`.
    """
    import torch
    lib = L.load()
    n = len(entries)
    arr = (L.Sweep * n)()
    keep, outs = [], []
    for i, e in enumerate(entries):
        prob = e["prob"]
        lam, plam = _dbl(e["lams"])
        nl = len(lam)
        x = torch.empty(nl * prob.n, dtype=torch.float64, device=e["b"].device)
        opts = L.SweepOpts(int(e.get("maxit", 100000)),
                           L.RLS_TOL_ABSOLUTE if e.get("tol_mode") == "absolute"
                           else L.RLS_TOL_RELATIVE,
                           int(e.get("poll_every", 32)),
                           1 if e.get("graph", True) else 0)
        res = np.zeros(nl)
        sem = np.zeros(nl)
        info = (L.SolveInfo * nl)()
        x0 = e.get("x0")
        w = arr[i]
        w.prob = prob._h
        w.b = _dptr(e["b"], "b", prob.m)
        w.lam = plam
        w.nlam = nl
        w.tol = float(e["tol"])
        w.opts = C.pointer(opts)
        w.x0 = None if x0 is None else _dptr(x0, "x0", nl * prob.n)
        w.x = _dptr(x, "x", nl * prob.n)
        w.resnorm = res.ctypes.data_as(C.POINTER(C.c_double))
        w.seminorm = sem.ctypes.data_as(C.POINTER(C.c_double))
        w.info = info
        keep += [lam, opts, res, sem, info]
        outs.append((x, res, sem, info, nl, prob.n))
    _check(lib.rls_solve_batch(arr, n, _stream()))
    result = []
    for x, res, sem, info, nl, npx in outs:
        inf = [dict(iters=i.iters, flags=i.flags, relres=i.relres,
                    relres_true=i.relres_true) for i in info]
        result.append((x.view(nl, npx), res, sem, inf))
    return result

