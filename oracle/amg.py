"""Oracle for classical (Ruge-Stueben) AMG coarsening of L^T D^2 L, the
operator-dependent interpolation of the paper's Sections 3.1 and 3.2.

Test infrastructure: only the tests use this module; the library never does.

  * strong_connections -- j strongly influences i when -k_ij exceeds theta
    times the largest negative off-diagonal of row i (theta = 0.25);
  * rs_split -- the two-pass C/F partition: a greedy maximal independent
    set of the strong-connection graph (measure = number of points that
    depend strongly on a point, raised for the unassigned strong
    neighbours of each new F point), then a second pass that turns F points
    into C points until every pair of strongly connected F points shares a
    strongly connected C point;
  * rs_interpolation -- the classical weights of Section 3.1,
    w_ij = -(k_ij + sum_{m in F_i^s} k_im k_mj / sum_{l in C_i} k_ml)
           / (k_ii + sum_{m in F_i^w} k_im);
  * AmgHierarchy -- the one-sided hierarchy of Section 3.2 with those P_k:
    P_k from the Galerkin operator M_k^T M_k, A_{k+1} = A_k P_k and
    M_{k+1} = M_k P_k, with the interface of the geometric Hierarchy so
    that the same V-cycles run on it.

Readings where the paper is silent: ties in the greedy selection go to the
lowest index; a point with no strong connections (neither way) becomes a C
point, so that constants stay exactly interpolable; the second pass follows
Ruge and Stueben (a first unshared strong F neighbour becomes a tentative
C point, a second one makes the point itself C); coarsening stops at
`max_coarse` unknowns or when a level would not shrink.
"""
import heapq

import numpy as np
import scipy.sparse as sp

from .multigrid import Hierarchy, SparseOp, colsumsq


def strong_connections(K, theta=0.25):
    """Boolean CSR S with S[i, j] = 1 when j strongly influences i."""
    K = sp.csr_matrix(K)
    n = K.shape[0]
    rows, cols = [], []
    for i in range(n):
        a, b = K.indptr[i], K.indptr[i + 1]
        js, vs = K.indices[a:b], K.data[a:b]
        off = js != i
        if not np.any(off):
            continue
        neg = -vs[off]
        top = neg.max()
        if top <= 0.0:
            continue
        keep = neg > theta * top
        rows += [i] * int(keep.sum())
        cols += list(js[off][keep])
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))


def rs_split(K, theta=0.25):
    """C/F labels (True = C) of the two-pass Ruge-Stueben coarsening."""
    S = strong_connections(K, theta)
    ST = S.T.tocsr()
    n = S.shape[0]
    UNSET, CPT, FPT = 0, 1, 2
    state = np.zeros(n, dtype=np.int8)
    lam = np.diff(ST.indptr).astype(np.int64)      # |S_i^T|
    for i in range(n):
        if lam[i] == 0 and S.indptr[i + 1] == S.indptr[i]:
            state[i] = CPT                          # isolated point
    heap = [(-int(lam[i]), i) for i in range(n) if state[i] == UNSET]
    heapq.heapify(heap)
    while heap:
        negl, i = heapq.heappop(heap)
        if state[i] != UNSET or -negl != lam[i]:
            continue                                # stale entry
        state[i] = CPT
        for j in ST.indices[ST.indptr[i]:ST.indptr[i + 1]]:
            if state[j] == UNSET:
                state[j] = FPT
                for k in S.indices[S.indptr[j]:S.indptr[j + 1]]:
                    if state[k] == UNSET:
                        lam[k] += 1
                        heapq.heappush(heap, (-int(lam[k]), k))
    state[state == UNSET] = FPT
    # second pass
    for i in range(n):
        if state[i] != FPT:
            continue
        Si = set(S.indices[S.indptr[i]:S.indptr[i + 1]])
        Ci = {j for j in Si if state[j] == CPT}
        tentative = None
        for j in sorted(Si):
            if state[j] != FPT:
                continue
            Sj = set(S.indices[S.indptr[j]:S.indptr[j + 1]])
            if Sj & Ci:
                continue
            if tentative is None:
                tentative = j
                Ci = Ci | {j}
            else:
                state[i] = CPT
                tentative = None
                break
        if tentative is not None:
            state[tentative] = CPT
    return state == CPT, S


def rs_interpolation(K, theta=0.25):
    """Classical interpolation P (n x n_c) for the Ruge-Stueben split."""
    K = sp.csr_matrix(K)
    is_c, S = rs_split(K, theta)
    n = K.shape[0]
    cidx = -np.ones(n, dtype=np.int64)
    cidx[is_c] = np.arange(int(is_c.sum()))
    rows, cols, vals = [], [], []
    for i in range(n):
        if is_c[i]:
            rows.append(i)
            cols.append(cidx[i])
            vals.append(1.0)
            continue
        a, b = K.indptr[i], K.indptr[i + 1]
        nbr = {int(j): float(v) for j, v in zip(K.indices[a:b], K.data[a:b])}
        kii = nbr.pop(i, 0.0)
        Si = set(S.indices[S.indptr[i]:S.indptr[i + 1]])
        Ci = [j for j in nbr if j in Si and is_c[j]]
        Fs = [m for m in nbr if m in Si and not is_c[m]]
        Fw = [m for m in nbr if m not in Si]
        den = kii + sum(nbr[m] for m in Fw)
        for j in Ci:
            num = nbr[j]
            for m in Fs:
                km = K.getrow(m)
                kmd = dict(zip(km.indices, km.data))
                tot = sum(kmd.get(l, 0.0) for l in Ci)
                num += nbr[m] * kmd.get(j, 0.0) / tot
            rows.append(i)
            cols.append(cidx[j])
            vals.append(-num / den)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, int(is_c.sum())))


class AmgHierarchy(Hierarchy):
    """One-sided hierarchy (Section 3.2) with Ruge-Stueben interpolation
    built from M_k^T M_k; same interface as the geometric Hierarchy."""

    def __init__(self, A, M, levels: int, theta=0.25, max_coarse=1024):
        self.levels = 1
        self.P = []
        self.A = [SparseOp(A.explicit())]
        self.M = [sp.csr_matrix(M)]
        while self.levels < levels and self.M[-1].shape[1] > max_coarse:
            Sk = (self.M[-1].T @ self.M[-1]).tocsr()
            P = rs_interpolation(Sk, theta)
            if P.shape[1] >= P.shape[0] or P.shape[1] == 0:
                break
            self.P.append(P)
            self.A.append(SparseOp(self.A[-1].A @ P))
            self.M.append((self.M[-1] @ P).tocsr())
            self.levels += 1
        self.diagA = [colsumsq(a) for a in self.A]
        self.diagM = [np.asarray(m.multiply(m).sum(axis=0)).ravel()
                      for m in self.M]
        # Gershgorin row sums: |A_k|^T |A_k| 1 bounds the rows of |A_k^T A_k|
        # (interpolation weights may be negative, so A_k need not be >= 0)
        self.rowabsA, self.rowabsM = [], []
        for a, m in zip(self.A, self.M):
            Aa = abs(sp.csr_matrix(a.A))
            ones = np.ones(Aa.shape[1])
            self.rowabsA.append(Aa.T @ (Aa @ ones))
            Sm = (m.T @ m).tocsr()
            self.rowabsM.append(np.asarray(abs(Sm).sum(axis=1)).ravel())
