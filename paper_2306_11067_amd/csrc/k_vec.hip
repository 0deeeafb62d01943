// Pointwise multigrid pieces: first smoothing step from a zero guess,
// restriction R = P^T, prolongation with correction, and the exact
// coarsest solve (Algorithm 1).
#include "common.h"

namespace rls {

// x = c2 f / diag(K), d = x: the first Chebyshev step from x = 0.
__global__ void k_jacobi_init(LevelGeom g, const double* __restrict__ lam2,
                              const int* __restrict__ slots,
                              const int* __restrict__ active,
                              const double* __restrict__ f, int f_shared,
                              const double* __restrict__ cheb, int cheb_stride,
                              double* __restrict__ x, double* __restrict__ d) {
    const int slot = slots ? slots[blockIdx.y] : (int)blockIdx.y;
    if (active && !active[slot]) return;
    const int64_t n = (int64_t)g.nv * g.nh;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int i = (int)(p % g.nv), j = (int)(p / g.nv);
    const double dg = g.gv.diag[i] * g.gh.diag[j] + lam2[slot] * g.S.c[p];
    const size_t o = (size_t)slot * n + p;
    const double v = cheb[(size_t)slot * cheb_stride + 1] * f[f_shared ? p : o] / dg;
    x[o] = v;
    d[o] = v;
}

// fc(I, J) = sum_{f} P(f, (I, J)) res(f): full weighting with R = P^T.
__global__ void k_restrict(int nvf, int nhf, int periodic,
                           const int* __restrict__ active,
                           const double* __restrict__ res,
                           double* __restrict__ fc) {
    const int slot = blockIdx.y;
    if (active && !active[slot]) return;
    const int nvc = nvf >> 1, nhc = nhf >> 1;
    const int64_t nc = (int64_t)nvc * nhc, nf = (int64_t)nvf * nhf;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nc) return;
    const int I = (int)(q % nvc), J = (int)(q / nvc);
    const double* r = res + (size_t)slot * nf;
    double s = 0.0;
    for (int b = -1; b <= 1; ++b) {
        int fj = 2 * J + b;
        if (!wrap_or_drop(fj, nhf, periodic)) continue;
        const double wj = interp_weight(fj, J, nhf, periodic);
        if (wj == 0.0) continue;
        double cs = 0.0;
        for (int a2 = -1; a2 <= 1; ++a2) {
            int fi = 2 * I + a2;
            if (!wrap_or_drop(fi, nvf, periodic)) continue;
            const double wi = interp_weight(fi, I, nvf, periodic);
            if (wi != 0.0) cs += wi * r[fi + (int64_t)nvf * fj];
        }
        s += wj * cs;
    }
    fc[(size_t)slot * nc + q] = s;
}

// Coarse points contributing to fine point f (at most two) and weights.
__device__ __forceinline__ int interp_sources_v(int f, int nf, int periodic,
                                              int* I, double* w) {
    const int nc = nf >> 1;
    if ((f & 1) == 0) { I[0] = f >> 1; w[0] = 1.0; return 1; }
    const int c = f >> 1;
    if (c + 1 < nc) { I[0] = c; I[1] = c + 1; w[0] = w[1] = 0.5; return 2; }
    if (periodic) { I[0] = c; I[1] = 0; w[0] = w[1] = 0.5; return 2; }
    I[0] = c; w[0] = 1.0; return 1;
}

// x(f) += sum_{I} P(f, I) ec(I).
__global__ void k_prolong_add(int nvf, int nhf, int periodic,
                              const int* __restrict__ active,
                              const double* __restrict__ ec,
                              double* __restrict__ x) {
    const int slot = blockIdx.y;
    if (active && !active[slot]) return;
    const int nvc = nvf >> 1, nhc = nhf >> 1;
    const int64_t nc = (int64_t)nvc * nhc, nf = (int64_t)nvf * nhf;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nf) return;
    const int fi = (int)(p % nvf), fj = (int)(p / nvf);
    int Ii[2], Jj[2];
    double wi[2], wj[2];
    const int ni = interp_sources_v(fi, nvf, periodic, Ii, wi);
    const int nj = interp_sources_v(fj, nhf, periodic, Jj, wj);
    const double* e = ec + (size_t)slot * nc;
    double s = 0.0;
    for (int b = 0; b < nj; ++b) {
        double cs = 0.0;
        for (int a2 = 0; a2 < ni; ++a2) cs += wi[a2] * e[Ii[a2] + (int64_t)nvc * Jj[b]];
        s += wj[b] * cs;
    }
    x[(size_t)slot * nf + p] += s;
}

// z = W^T (W f) with W = L^{-1}, K_c = L L^T: the exact coarsest solve.
// W row-major at Winv[slot], W^T (row-major) right after it.
__global__ void __launch_bounds__(1024)
k_coarse_solve(const double* __restrict__ Wall, int n,
               const int* __restrict__ slots, const int* __restrict__ active,
               const double* __restrict__ f, double* __restrict__ z) {
    extern __shared__ double sh[];
    const int slot = slots ? slots[blockIdx.x] : (int)blockIdx.x;
    if (active && !active[slot]) return;
    const double* W = Wall + (size_t)slot * 2 * n * n;
    const double* Wt = W + (size_t)n * n;   // Wt[c*n + i] = W(i, c)
    double* fs = sh;
    double* ys = sh + n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) fs[i] = f[(size_t)slot * n + i];
    __syncthreads();
    // y(i) = sum_{m <= i} W(i, m) f(m); W(i, m) = Wt[m*n + i] (coalesced in i)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double s = 0.0;
        for (int m = 0; m <= i; ++m) s += Wt[(size_t)m * n + i] * fs[m];
        ys[i] = s;
    }
    __syncthreads();
    // z(c) = sum_{m >= c} W(m, c) y(m); W(m, c) = W[m*n + c] (coalesced in c)
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        double s = 0.0;
        for (int m = c; m < n; ++m) s += W[(size_t)m * n + c] * ys[m];
        z[(size_t)slot * n + c] = s;
    }
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_jacobi_init(const LevelGeom& g, int nslot, const double* lam2,
                        const int* slots, const int* active, const double* f,
                        int f_shared, const double* cheb, int cheb_stride,
                        double* x, double* d, hipStream_t s) {
    const int64_t n = (int64_t)g.nv * g.nh;
    hipLaunchKernelGGL(k_jacobi_init, dim3(nblk(n, 256), nslot), dim3(256), 0,
                       s, g, lam2, slots, active, f, f_shared, cheb, cheb_stride,
                       x, d);
}

void launch_restrict(const LevelGeom& fine, const LevelGeom& coarse, int nslot,
                     const int* active, const double* res, double* fc,
                     hipStream_t s) {
    const int64_t nc = (int64_t)coarse.nv * coarse.nh;
    hipLaunchKernelGGL(k_restrict, dim3(nblk(nc, 256), nslot), dim3(256), 0, s,
                       fine.nv, fine.nh, fine.S.periodic, active, res, fc);
}

void launch_prolong_add(const LevelGeom& fine, const LevelGeom& coarse,
                        int nslot, const int* active, const double* ec,
                        double* x, hipStream_t s) {
    (void)coarse;
    const int64_t nf = (int64_t)fine.nv * fine.nh;
    hipLaunchKernelGGL(k_prolong_add, dim3(nblk(nf, 256), nslot), dim3(256), 0,
                       s, fine.nv, fine.nh, fine.S.periodic, active, ec, x);
}

void launch_coarse_solve(const double* Wall, int n, int nslot,
                         const int* slots, const int* active, const double* f,
                         double* z, hipStream_t s) {
    const int threads = n >= 1024 ? 1024 : ((n + 63) / 64) * 64;
    hipLaunchKernelGGL(k_coarse_solve, dim3(nslot), dim3(threads),
                       2 * n * sizeof(double), s, Wall, n, slots, active, f, z);
}

}  // namespace rls
