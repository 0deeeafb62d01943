"""Helpers shared by the GPU tests (marshalling between numpy and torch)."""
import numpy as np


def cuda_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def planes_from_sparse(S, nv, nh, periodic):
    """Five-plane layout of a 9-point operator given as a sparse matrix:
    centre, (i+1, j), (i, j+1), (i+1, j+1), (i-1, j+1)."""
    S = S.tocsr()
    n = nv * nh
    out = np.zeros((5, n))
    offs = [(0, 0), (1, 0), (0, 1), (1, 1), (-1, 1)]
    for j in range(nh):
        for i in range(nv):
            p = i + nv * j
            for t, (di, dj) in enumerate(offs):
                ii, jj = i + di, j + dj
                if periodic:
                    ii %= nv
                    jj %= nh
                elif not (0 <= ii < nv and 0 <= jj < nh):
                    continue
                out[t, p] = S[p, ii + nv * jj]
    return out


def band_from_dense(G, periodic):
    """Band rows (n, 2bw+1) of a dense banded matrix; bw inferred."""
    n = G.shape[0]
    nz = np.nonzero(G)
    bw = 0
    for r, c in zip(*nz):
        d = c - r
        if periodic:
            d = (d + n // 2) % n - n // 2
        bw = max(bw, abs(d))
    out = np.zeros((n, 2 * bw + 1))
    for r in range(n):
        for k in range(-bw, bw + 1):
            c = r + k
            if periodic:
                c %= n
            elif not 0 <= c < n:
                continue
            out[r, k + bw] = G[r, c]
    return out, bw
