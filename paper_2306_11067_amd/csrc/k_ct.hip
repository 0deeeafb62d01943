// Level operator K_k(lambda) v = A_k^T (A_k v) + lambda^2 S_k v for a sparse
// (tomography) forward operator: the two-stage product of the paper's
// Section 3.2 with the one-sided A_k = A P_1 ... P_k stored as CSR (and its
// transpose), batched over lambda slots.  One application is
//   prologue (form v: p update, Jacobi start, coarse correction) ->
//   y = A_k v -> t = A_k^T y -> stencil term and epilogue
// (the same prologues and epilogues as the separable-blur kernel), plus a
// full-weighting restriction for the restriction epilogue.
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "pcg_ctl.h"

namespace rls {

constexpr int CT_THREADS = 256;

template <class R>
__device__ __forceinline__ R ct_diag(const LevelGeomT<R>& g, R l2, int64_t p) {
    return g.ct.diag[p] + l2 * g.S.c[p];
}

// (P e)(fi, fj) for the coarse vector e of size (nvf/2) x (nhf/2).
template <class R>
__device__ __forceinline__ R ct_prolong(const R* __restrict__ e, int fi, int fj,
                                        int nvf, int nhf, int periodic) {
    const int nvc = nvf >> 1, nhc = nhf >> 1;
    R s = R(0);
    for (int b = -1; b <= 1; ++b) {
        int J = (fj >> 1) + b;
        if (!wrap_or_drop(J, nhc, periodic)) continue;
        const R wj = (R)interp_weight(fj, J, nhf, periodic);
        if (wj == R(0)) continue;
        R cs = R(0);
        for (int a = -1; a <= 1; ++a) {
            int I = (fi >> 1) + a;
            if (!wrap_or_drop(I, nvc, periodic)) continue;
            const R wi = (R)interp_weight(fi, I, nvf, periodic);
            if (wi != R(0)) cs += wi * e[I + (int64_t)nvc * J];
        }
        s += wj * cs;
    }
    return s;
}

// v on every point of the slot (PUPDATE writes p_new, the others a temp).
template <int PRO, class R>
__global__ void __launch_bounds__(CT_THREADS)
k_ct_prologue(ApplyArgsT<R> a, R* vout) {
    __shared__ double red[CT_THREADS];
    const int z = blockIdx.y;
    const int slot = a.slots ? a.slots[z] : z;
    if (a.active && !a.active[slot]) return;
    const LevelGeomT<R>& g = a.g;
    const int nv = g.nv, nh = g.nh;
    const int64_t n = (int64_t)nv * nh;
    const bool lead = blockIdx.x == 0;
    double beta = 0.0;
    if (PRO == PRO_PUPDATE) {
        if (!pcg_beta<CT_THREADS>(a.st, a.active_w, slot, a.part_rz, a.nrz,
                                  a.parity, a.flex ? a.part_zq : nullptr, lead,
                                  red, beta))
            return;
    }
    if (a.gate) {
        if (!pcg_gate<CT_THREADS>(a.st, a.active_w, slot, a.part_rr, a.nrr,
                                  lead, red))
            return;
    }
    const int64_t p = (int64_t)blockIdx.x * CT_THREADS + threadIdx.x;
    if (p >= n) return;
    const size_t so = (size_t)slot * n;
    const R l2 = (R)a.lam2[slot];
    R v;
    if (PRO == PRO_PUPDATE) {
        const R po = beta == 0.0 ? R(0) : a.pold[so + p];
        v = a.in[so + p] + (R)beta * po;
    } else {
        const int i = (int)(p % nv), j = (int)(p / nv);
        v = R(0);
        if (PRO == PRO_JACOBI || PRO == PRO_PROLONG_JAC) {
            const R cj = (R)a.cheb_first[(size_t)slot * a.cheb_stride + 1];
            v = cj * a.f[(a.f_shared ? 0 : so) + p] / ct_diag(g, l2, p);
        }
        if (PRO == PRO_PROLONG) v = a.in[so + p];
        if (PRO == PRO_PROLONG || PRO == PRO_PROLONG_JAC)
            v += ct_prolong(a.ec + (size_t)slot * (n >> 2), i, j, nv, nh,
                            g.S.periodic);
    }
    vout[so + p] = v;
}

// kv = t + lambda^2 S v at every point, then the epilogue.
template <int PRO, int EPI, class R>
__global__ void __launch_bounds__(CT_THREADS)
k_ct_epilogue(ApplyArgsT<R> a, const R* __restrict__ vs) {
    __shared__ double red[CT_THREADS];
    const int z = blockIdx.y;
    const int slot = a.slots ? a.slots[z] : z;
    if (a.active && !a.active[slot]) return;
    const LevelGeomT<R>& g = a.g;
    const int nv = g.nv, nh = g.nh, per = g.S.periodic;
    const int64_t n = (int64_t)nv * nh;
    const size_t so = (size_t)slot * n;
    const int64_t p = (int64_t)blockIdx.x * CT_THREADS + threadIdx.x;
    double dot = 0.0;
    if (p < n) {
        const R l2 = (R)a.lam2[slot];
        const int i = (int)(p % nv), j = (int)(p / nv);
        const R* v = vs + so;
        auto at = [&](int ii, int jj) { return v[ii + (int64_t)nv * jj]; };
        int im = i - 1, ip = i + 1, jm = j - 1, jp = j + 1;
        const bool okim = wrap_or_drop(im, nv, per), okip = wrap_or_drop(ip, nv, per);
        const bool okjm = wrap_or_drop(jm, nh, per), okjp = wrap_or_drop(jp, nh, per);
        const R vc = v[p];
        R sv = g.S.c[p] * vc;
        if (okip) sv += g.S.cn[p] * at(ip, j);
        if (okim) sv += g.S.cn[im + (int64_t)nv * j] * at(im, j);
        if (okjp) sv += g.S.ce[p] * at(i, jp);
        if (okjm) sv += g.S.ce[i + (int64_t)nv * jm] * at(i, jm);
        if (g.S.nine) {
            if (okip && okjp) sv += g.S.cne[p] * at(ip, jp);
            if (okim && okjm) sv += g.S.cne[im + (int64_t)nv * jm] * at(im, jm);
            if (okim && okjp) sv += g.S.cse[p] * at(im, jp);
            if (okip && okjm) sv += g.S.cse[ip + (int64_t)nv * jm] * at(ip, jm);
        }
        const R kv = g.ct.t[so + p] + l2 * sv;
        if (EPI == EPI_STORE) {
            a.out[so + p] = kv;
        } else if (EPI == EPI_DOT) {
            a.out[so + p] = kv;
            dot = (double)vc * (double)kv;
        } else {
            const R f = a.f[(a.f_shared ? 0 : so) + p];
            if (EPI == EPI_RESID) {
                a.out[so + p] = f - kv;
            } else if (EPI == EPI_RESTRICT) {
                g.ct.res[so + p] = f - kv;
            } else {   // EPI_CHEB
                const double* cc = a.cheb + (size_t)slot * a.cheb_stride;
                const R dprev = PRO == PRO_JACOBI ? vc : a.d[so + p];
                const R dn = (R)cc[0] * dprev + (R)cc[1] * (f - kv) / ct_diag(g, l2, p);
                a.d[so + p] = dn;
                const R xn = vc + dn;
                a.out[so + p] = xn;
                if (a.dot) dot = (double)f * (double)xn;
            }
        }
    }
    if (EPI == EPI_DOT || (EPI == EPI_CHEB && a.dot)) {
        const double s = block_sum<CT_THREADS>(dot, red);
        if (threadIdx.x == 0) a.part[(size_t)slot * a.part_stride + blockIdx.x] = s;
    }
}

// fc(I, J) = sum_f P(f, (I, J)) res(f) (full weighting, R = P^T).
template <class R>
__global__ void __launch_bounds__(CT_THREADS)
k_ct_restrict(int nvf, int nhf, int per, const int* slots, const int* active,
              const R* __restrict__ res, R* __restrict__ fc) {
    const int z = blockIdx.y;
    const int slot = slots ? slots[z] : z;
    if (active && !active[slot]) return;
    const int nvc = nvf >> 1, nhc = nhf >> 1;
    const int64_t nc = (int64_t)nvc * nhc, nf = (int64_t)nvf * nhf;
    const int64_t e = (int64_t)blockIdx.x * CT_THREADS + threadIdx.x;
    if (e >= nc) return;
    const int I = (int)(e % nvc), J = (int)(e / nvc);
    const R* r = res + (size_t)slot * nf;
    R s = R(0);
    for (int b = -1; b <= 1; ++b) {
        int fj = 2 * J + b;
        if (!wrap_or_drop(fj, nhf, per)) continue;
        const R wj = (R)interp_weight(fj, J, nhf, per);
        if (wj == R(0)) continue;
        R cs = R(0);
        for (int a2 = -1; a2 <= 1; ++a2) {
            int fi = 2 * I + a2;
            if (!wrap_or_drop(fi, nvf, per)) continue;
            const R wi = (R)interp_weight(fi, I, nvf, per);
            if (wi != R(0)) cs += wi * r[fi + (int64_t)nvf * fj];
        }
        s += wj * cs;
    }
    fc[(size_t)slot * nc + e] = s;
}

template <int PRO, int EPI, class R>
static void ct_apply(const ApplyArgsT<R>& a, hipStream_t s) {
    const LevelGeomT<R>& g = a.g;
    const CsrDevT<R>& c = g.ct;
    const int64_t n = (int64_t)g.nv * g.nh;
    const dim3 grid((unsigned)((n + CT_THREADS - 1) / CT_THREADS), a.nslot);
    const R* vs = a.in;
    if (PRO != PRO_PLAIN) {
        R* vo = PRO == PRO_PUPDATE ? a.pnew : c.v;
        hipLaunchKernelGGL((k_ct_prologue<PRO, R>), grid, dim3(CT_THREADS), 0, s,
                           a, vo);
        vs = vo;
    }
    launch_spmv<R, R, R>(c.rp, c.ci, c.va, c.m, n, vs, 0, c.m, c.y, a.nslot,
                         a.slots, a.active, s);
    launch_spmv<R, R, R>(c.rpt, c.cit, c.vat, n, c.m, c.y, 0, n, c.t, a.nslot,
                         a.slots, a.active, s);
    hipLaunchKernelGGL((k_ct_epilogue<PRO, EPI, R>), grid, dim3(CT_THREADS), 0,
                       s, a, vs);
    if (EPI == EPI_RESTRICT) {
        const int64_t nc = n / 4;
        hipLaunchKernelGGL((k_ct_restrict<R>),
                           dim3((unsigned)((nc + CT_THREADS - 1) / CT_THREADS),
                                a.nslot),
                           dim3(CT_THREADS), 0, s, g.nv, g.nh, g.S.periodic,
                           a.slots, a.active, c.res, a.fc);
    }
}

#define RLS_CT_VARIANTS(X)            \
    X(PRO_PUPDATE, EPI_DOT)           \
    X(PRO_JACOBI, EPI_CHEB)           \
    X(PRO_JACOBI, EPI_RESTRICT)       \
    X(PRO_PROLONG, EPI_CHEB)          \
    X(PRO_PROLONG_JAC, EPI_CHEB)      \
    X(PRO_PLAIN, EPI_STORE)           \
    X(PRO_PLAIN, EPI_DOT)             \
    X(PRO_PLAIN, EPI_RESID)           \
    X(PRO_PLAIN, EPI_RESTRICT)        \
    X(PRO_PLAIN, EPI_CHEB)

template <class R>
static void ct_dispatch(int pro, int epi, const ApplyArgsT<R>& a,
                        hipStream_t s) {
#define RLS_CT(P, E) \
    if (pro == P && epi == E) { ct_apply<P, E, R>(a, s); return; }
    RLS_CT_VARIANTS(RLS_CT)
#undef RLS_CT
    std::fprintf(stderr, "rls: no sparse level operator for prologue %d, "
                         "epilogue %d\n", pro, epi);
    std::abort();
}

void launch_ct_apply(int pro, int epi, const ApplyArgsT<double>& a,
                     hipStream_t s) {
    ct_dispatch(pro, epi, a, s);
}
void launch_ct_apply(int pro, int epi, const ApplyArgsT<float>& a,
                     hipStream_t s) {
    ct_dispatch(pro, epi, a, s);
}

int ct_parts(int64_t n) { return (int)((n + CT_THREADS - 1) / CT_THREADS); }

}  // namespace rls
