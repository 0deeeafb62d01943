// Coarse tail of the V-cycle in one workgroup per lambda slot.
//
// The levels whose grids hold at most TAIL_MAX_POINTS unknowns, down to
// and including the coarsest one, are processed by a single 1024-thread
// workgroup with every vector in LDS and workgroup barriers between the
// steps of Algorithm 1 (smoothing, residual, restriction, exact coarsest
// solve, prolongation and correction, smoothing).  On these grids a kernel
// launch per step would cost more than the arithmetic; here the whole tail
// is one launch.  The arithmetic is the same as on the tiled levels: the
// separable Gram bands plus lambda^2 times the 9-point Galerkin stencil,
// Jacobi-scaled Chebyshev steps, R = P^T, and z = W^T (W f) with
// W = L^{-1} from the Cholesky factor of the coarsest matrix.
#include "common.h"
#include "pcg_ctl.h"

namespace rls {

constexpr int TAIL_THREADS = 1024;

struct TailScratch {
    double* t;    // temp (max(n_first, TAIL_THREADS))
    double* xb;   // ping-pong partner of X[k]
    double* d;    // Chebyshev direction
    double* res;  // residual
};

__device__ __forceinline__ int tail_wrap(int j, int n, int periodic, bool& ok) {
    ok = true;
    if (j >= 0 && j < n) return j;
    if (!periodic) { ok = false; return 0; }
    j %= n;
    return j < 0 ? j + n : j;
}

__device__ __forceinline__ double tail_diag(const TailLevel& L, double l2,
                                            int i, int j, int p) {
    return L.gv.diag[i] * L.gh.diag[j] + l2 * L.S.c[p];
}

// out(p) = (K v)(p) for every point, handed to `epi(p, kv)`.  Ends with a
// barrier; v must not be written by `epi`.
template <class Epi>
__device__ void tail_apply(const TailLevel& L, double l2, int per,
                           const double* v, double* t, Epi epi) {
    const int nv = L.nv, nh = L.nh, n = nv * nh;
    const int wv = 2 * L.gv.bw + 1, wh = 2 * L.gh.bw + 1;
    for (int p = threadIdx.x; p < n; p += TAIL_THREADS) {
        const int i = p % nv, j = p / nv;
        double s = 0.0;
        for (int k = -L.gv.bw; k <= L.gv.bw; ++k) {
            bool ok;
            const int ii = tail_wrap(i + k, nv, per, ok);
            if (ok) s += L.gv.table[i * wv + k + L.gv.bw] * v[ii + nv * j];
        }
        t[p] = s;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < n; p += TAIL_THREADS) {
        const int i = p % nv, j = p / nv;
        double kv = 0.0;
        for (int k = -L.gh.bw; k <= L.gh.bw; ++k) {
            bool ok;
            const int jj = tail_wrap(j + k, nh, per, ok);
            if (ok) kv += L.gh.table[j * wh + k + L.gh.bw] * t[i + nv * jj];
        }
        bool oim, ojm, oip, ojp;
        const int im = tail_wrap(i - 1, nv, per, oim);
        const int ip = tail_wrap(i + 1, nv, per, oip);
        const int jm = tail_wrap(j - 1, nh, per, ojm);
        const int jp = tail_wrap(j + 1, nh, per, ojp);
        double sv = L.S.c[p] * v[p];
        if (oip) sv += L.S.cn[p] * v[ip + nv * j];
        if (oim) sv += L.S.cn[im + nv * j] * v[im + nv * j];
        if (ojp) sv += L.S.ce[p] * v[i + nv * jp];
        if (ojm) sv += L.S.ce[i + nv * jm] * v[i + nv * jm];
        if (L.S.nine) {
            if (oip && ojp) sv += L.S.cne[p] * v[ip + nv * jp];
            if (oim && ojm) sv += L.S.cne[im + nv * jm] * v[im + nv * jm];
            if (oim && ojp) sv += L.S.cse[p] * v[im + nv * jp];
            if (oip && ojm) sv += L.S.cse[ip + nv * jm] * v[ip + nv * jm];
        }
        epi(p, kv + l2 * sv);
    }
    __syncthreads();
}

// nu Chebyshev steps on level L for K x = f; from zero when `from_zero`,
// else from x.  The result is left in x (LDS).
__device__ void tail_smooth(const TailLevel& L, double l2, int per, int nu,
                            const double* cheb, bool from_zero, double* x,
                            const double* f, TailScratch& sc) {
    const int nv = L.nv, n = L.nv * L.nh;
    double* cur = x;
    double* oth = sc.xb;
    int st = 0;
    if (from_zero) {
        const double c2 = cheb[1];
        for (int p = threadIdx.x; p < n; p += TAIL_THREADS) {
            const double v = c2 * f[p] / tail_diag(L, l2, p % nv, p / nv, p);
            cur[p] = v;
            sc.d[p] = v;
        }
        __syncthreads();
        st = 1;
    }
    for (; st < nu; ++st) {
        const double c1 = cheb[2 * st], c2 = cheb[2 * st + 1];
        double* in = cur;
        double* out = oth;
        tail_apply(L, l2, per, in, sc.t, [&](int p, double kv) {
            const double dn = c1 * sc.d[p] +
                              c2 * (f[p] - kv) / tail_diag(L, l2, p % nv, p / nv, p);
            sc.d[p] = dn;
            out[p] = in[p] + dn;
        });
        cur = out;
        oth = in;
    }
    if (cur != x) {
        for (int p = threadIdx.x; p < n; p += TAIL_THREADS) x[p] = cur[p];
        __syncthreads();
    }
}

template <class IO>
__global__ void __launch_bounds__(TAIL_THREADS) k_tail(TailArgsT<IO> a) {
    extern __shared__ double lds[];
    __shared__ double red[TAIL_THREADS];
    const int slot = a.slots ? a.slots[blockIdx.x] : (int)blockIdx.x;
    if (a.active && !a.active[slot]) return;
    if (a.gate) {
        // one workgroup per slot: it leads
        if (!pcg_gate<TAIL_THREADS>(a.st, a.active_w, slot, a.part_rr, a.nrr,
                                    true, red))
            return;
    }
    const int nl = a.nlev;
    const int per = a.periodic;
    const double l2 = a.lam2[slot];
    // LDS carve-up: X[k], F[k] per level, then the scratch vectors
    double* X[TAIL_MAX_LEVELS];
    double* F[TAIL_MAX_LEVELS];
    double* q = lds;
    for (int k = 0; k < nl; ++k) {
        const int nk = a.lev[k].nv * a.lev[k].nh;
        X[k] = q;
        q += nk;
        F[k] = q;
        q += nk;
    }
    const int n0 = a.lev[0].nv * a.lev[0].nh;
    const int nt = n0 > TAIL_THREADS ? n0 : TAIL_THREADS;
    TailScratch sc;
    sc.t = q;
    sc.xb = q + nt;
    sc.d = q + 2 * nt;
    sc.res = q + 3 * nt;

    for (int p = threadIdx.x; p < n0; p += TAIL_THREADS)
        F[0][p] = Cvt<double, IO>::in(a.f[(size_t)slot * n0 + p]);
    __syncthreads();

    // down: smooth, residual, restrict
    for (int k = 0; k + 1 < nl; ++k) {
        const TailLevel& L = a.lev[k];
        const double* cheb = L.cheb + (size_t)slot * a.cheb_stride;
        tail_smooth(L, l2, per, L.nu, cheb, true, X[k], F[k], sc);
        const double* fk = F[k];
        double* res = sc.res;
        tail_apply(L, l2, per, X[k], sc.t,
                   [&](int p, double kv) { res[p] = fk[p] - kv; });
        const int nvf = L.nv, nhf = L.nh, nvc = nvf >> 1, nc = nvc * (nhf >> 1);
        for (int e = threadIdx.x; e < nc; e += TAIL_THREADS) {
            const int I = e % nvc, J = e / nvc;
            double s = 0.0;
            for (int b = -1; b <= 1; ++b) {
                int fj = 2 * J + b;
                if (!wrap_or_drop(fj, nhf, per)) continue;
                const double wj = interp_weight(fj, J, nhf, per);
                if (wj == 0.0) continue;
                double cs = 0.0;
                for (int a2 = -1; a2 <= 1; ++a2) {
                    int fi = 2 * I + a2;
                    if (!wrap_or_drop(fi, nvf, per)) continue;
                    const double wi = interp_weight(fi, I, nvf, per);
                    if (wi != 0.0) cs += wi * res[fi + nvf * fj];
                }
                s += wj * cs;
            }
            F[k + 1][e] = s;
        }
        __syncthreads();
    }

    // coarsest: X = W^T (W F), W = L^{-1} of K_c = L L^T
    {
        const int nc = a.lev[nl - 1].nv * a.lev[nl - 1].nh;
        const double* W = a.W + (size_t)slot * 2 * nc * nc;
        const double* Wt = W + (size_t)nc * nc;
        int tpr = TAIL_THREADS / nc;            // threads per row (power of 2)
        if (tpr < 1) tpr = 1;
        if (tpr > 64) tpr = 64;
        double* t = sc.t;
        const double* fin = F[nl - 1];
        double* y = sc.res;
        for (int pass = 0; pass < 2; ++pass) {
            const double* M = pass == 0 ? W : Wt;   // rows of W, then of W^T
            const double* src = pass == 0 ? fin : y;
            for (int e = threadIdx.x; e < nc * tpr; e += TAIL_THREADS) {
                const int row = e / tpr, lane = e - row * tpr;
                double s = 0.0;
                for (int m = lane; m < nc; m += tpr) s += M[(size_t)row * nc + m] * src[m];
                t[e] = s;
            }
            __syncthreads();
            double* dst = pass == 0 ? y : X[nl - 1];
            for (int row = threadIdx.x; row < nc; row += TAIL_THREADS) {
                double s = 0.0;
                for (int l = 0; l < tpr; ++l) s += t[row * tpr + l];
                dst[row] = s;
            }
            __syncthreads();
        }
    }

    // up: prolong and correct, smooth
    for (int k = nl - 2; k >= 0; --k) {
        const TailLevel& L = a.lev[k];
        const int nvf = L.nv, nhf = L.nh, nvc = nvf >> 1, nf = nvf * nhf;
        const double* e = X[k + 1];
        for (int p = threadIdx.x; p < nf; p += TAIL_THREADS) {
            const int fi = p % nvf, fj = p / nvf;
            double s = 0.0;
            for (int b = -1; b <= 1; ++b) {
                int J = (fj >> 1) + b;
                if (!wrap_or_drop(J, nhf >> 1, per)) continue;
                const double wj = interp_weight(fj, J, nhf, per);
                if (wj == 0.0) continue;
                double cs = 0.0;
                for (int a2 = -1; a2 <= 1; ++a2) {
                    int I = (fi >> 1) + a2;
                    if (!wrap_or_drop(I, nvc, per)) continue;
                    const double wi = interp_weight(fi, I, nvf, per);
                    if (wi != 0.0) cs += wi * e[I + nvc * J];
                }
                s += wj * cs;
            }
            X[k][p] += s;
        }
        __syncthreads();
        const double* cheb = L.cheb + (size_t)slot * a.cheb_stride;
        tail_smooth(L, l2, per, L.nu, cheb, false, X[k], F[k], sc);
    }

    // store z (and r . z partials when the tail is the whole cycle)
    double dot = 0.0;
    for (int p = threadIdx.x; p < n0; p += TAIL_THREADS) {
        const double zv = X[0][p];
        a.z[(size_t)slot * n0 + p] = Cvt<double, IO>::out(zv);
        dot += F[0][p] * zv;
    }
    if (a.dot) {
        const double s = block_sum<TAIL_THREADS>(dot, red);
        for (int t2 = threadIdx.x; t2 < a.part_stride; t2 += TAIL_THREADS)
            a.part[(size_t)slot * a.part_stride + t2] = t2 == 0 ? s : 0.0;
    }
}

template <class IO>
size_t tail_lds_bytes(const TailArgsT<IO>& a) {
    size_t d = 0;
    for (int k = 0; k < a.nlev; ++k) d += 2 * (size_t)a.lev[k].nv * a.lev[k].nh;
    const size_t n0 = (size_t)a.lev[0].nv * a.lev[0].nh;
    d += 4 * (n0 > (size_t)TAIL_THREADS ? n0 : (size_t)TAIL_THREADS);
    return d * sizeof(double);
}
template size_t tail_lds_bytes(const TailArgsT<double>&);
template size_t tail_lds_bytes(const TailArgsT<float>&);
template size_t tail_lds_bytes(const TailArgsT<bf16>&);

template <class IO>
static void tail_impl(const TailArgsT<IO>& a, int nslot, hipStream_t s) {
    static bool configured = false;
    if (!configured) {
        hipFuncAttributes attr;
        size_t stat = 0;
        if (hipFuncGetAttributes(&attr, (const void*)k_tail<IO>) == hipSuccess)
            stat = attr.sharedSizeBytes;
        (void)hipFuncSetAttribute((const void*)k_tail<IO>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(160 * 1024 - stat));
        (void)hipGetLastError();
        configured = true;
    }
    hipLaunchKernelGGL(k_tail<IO>, dim3(nslot), dim3(TAIL_THREADS),
                       tail_lds_bytes(a), s, a);
}

void launch_tail(const TailArgsT<double>& a, int nslot, hipStream_t s) {
    tail_impl(a, nslot, s);
}
void launch_tail(const TailArgsT<float>& a, int nslot, hipStream_t s) {
    tail_impl(a, nslot, s);
}
void launch_tail(const TailArgsT<bf16>& a, int nslot, hipStream_t s) {
    tail_impl(a, nslot, s);
}

}  // namespace rls
