// Level operator K_k(lambda) v = (G_h (x) G_v) v + lambda^2 S_k v, batched
// over lambda, with fused prologue (how v is formed) and epilogue (what is
// done with K v).  One workgroup computes a TILE_Y x TILE_X output tile of
// one lambda slot:
//   1. load v on the tile plus a halo of max(bw, 1) into LDS (index map of
//      the Gram band supplies wrap / reflection / zero outside the grid);
//   2. vertical pass of G_v over the tile rows for every loaded column;
//   3. horizontal pass of G_h;
//   4. add lambda^2 times the 9-point stencil S_k from the LDS tile;
//   5. epilogue.
// This is the "two-stage" level product of the paper's Section 3.2: for the
// blur the products with A_k and A_k^T collapse into the separable Gram, and
// M_k^T M_k is the Galerkin stencil of L^T D^2 L.
#include "common.h"

namespace rls {

__device__ __forceinline__ double band_coeff(const BandDev& b, int r, int k) {
    return b.uniform ? b.taps[k + b.bw]
                     : b.table[(size_t)r * (2 * b.bw + 1) + k + b.bw];
}

template <int PRO, int EPI>
__global__ void __launch_bounds__(APPLY_THREADS) k_apply(ApplyArgs a) {
    extern __shared__ double lds[];
    const int slot = blockIdx.z;
    if (a.active && !a.active[slot]) return;
    const LevelGeom& g = a.g;
    const int nv = g.nv, nh = g.nh;
    const int64_t n = (int64_t)nv * nh;
    const int i0 = blockIdx.x * TILE_Y, j0 = blockIdx.y * TILE_X;
    const int bwv = g.gv.bw, bwh = g.gh.bw;
    const int hv = bwv > 1 ? bwv : 1, hh = bwh > 1 ? bwh : 1;
    const int RY = TILE_Y + 2 * hv;
    const int SY = RY | 1;
    const int CX = TILE_X + 2 * hh;
    const int SO = TILE_Y + 1;
    double* vin = lds;
    double* vt = lds + CX * SY;
    const double* src = a.in + (size_t)slot * n;
    const double l2 = a.lam2[slot];
    double beta = 0.0;
    if (PRO == PRO_PUPDATE) beta = a.beta[slot];

    // 1. load (with prologue)
    for (int e = threadIdx.x; e < CX * RY; e += APPLY_THREADS) {
        const int jj = e / RY, ii = e - jj * RY;
        const int ui = i0 - hv + ii, uj = j0 - hh + jj;
        bool okv, okh;
        const int gi = map_index(ui, nv, g.gv.map, okv);
        const int gj = map_index(uj, nh, g.gh.map, okh);
        double v = 0.0;
        if (okv && okh) {
            const int64_t p = gi + (int64_t)nv * gj;
            if (PRO == PRO_PLAIN) {
                v = src[p];
            } else {
                const double po = beta == 0.0 ? 0.0 : a.pold[(size_t)slot * n + p];
                v = src[p] + beta * po;
                const bool own = ii >= hv && ii < hv + TILE_Y && jj >= hh &&
                                 jj < hh + TILE_X && ui < nv && uj < nh;
                if (own) a.pnew[(size_t)slot * n + p] = v;
            }
        }
        vin[jj * SY + ii] = v;
    }
    __syncthreads();

    // 2. vertical pass: vt(ii, jj) = sum_k Gv(i0+ii, k) vin(ii+hv+k, jj)
    for (int e = threadIdx.x; e < TILE_Y * CX; e += APPLY_THREADS) {
        const int jj = e / TILE_Y, ii = e - jj * TILE_Y;
        const int gi = i0 + ii;
        double s = 0.0;
        if (gi < nv) {
            const double* col = vin + jj * SY + ii + hv;
            for (int k = -bwv; k <= bwv; ++k) s += band_coeff(g.gv, gi, k) * col[k];
        }
        vt[jj * SO + ii] = s;
    }
    __syncthreads();

    // 3.-5. horizontal pass, stencil, epilogue
    double dot = 0.0;
    for (int e = threadIdx.x; e < TILE_Y * TILE_X; e += APPLY_THREADS) {
        const int jo = e / TILE_Y, ii = e - jo * TILE_Y;
        const int gi = i0 + ii, gj = j0 + jo;
        if (gi >= nv || gj >= nh) continue;
        double kv = 0.0;
        for (int k = -bwh; k <= bwh; ++k)
            kv += band_coeff(g.gh, gj, k) * vt[(jo + hh + k) * SO + ii];
        // stencil
        const double* vc = vin + (jo + hh) * SY + ii + hv;   // v(gi, gj)
        const int64_t p = gi + (int64_t)nv * gj;
        const int per = g.S.periodic;
        int im = gi - 1, jm = gj - 1, ip = gi + 1;
        const bool okim = wrap_or_drop(im, nv, per);
        const bool okjm = wrap_or_drop(jm, nh, per);
        const bool okip = wrap_or_drop(ip, nv, per);
        double sv = g.S.c[p] * vc[0];
        sv += g.S.cn[p] * vc[1];
        if (okim) sv += g.S.cn[im + (int64_t)nv * gj] * vc[-1];
        sv += g.S.ce[p] * vc[SY];
        if (okjm) sv += g.S.ce[gi + (int64_t)nv * jm] * vc[-SY];
        if (g.S.nine) {
            sv += g.S.cne[p] * vc[SY + 1];
            if (okim && okjm) sv += g.S.cne[im + (int64_t)nv * jm] * vc[-SY - 1];
            sv += g.S.cse[p] * vc[SY - 1];
            if (okip && okjm) sv += g.S.cse[ip + (int64_t)nv * jm] * vc[-SY + 1];
        }
        kv += l2 * sv;
        const double v = vc[0];
        const size_t o = (size_t)slot * n + p;
        if (EPI == EPI_STORE) {
            a.out[o] = kv;
        } else if (EPI == EPI_DOT) {
            a.out[o] = kv;
            dot += v * kv;
        } else if (EPI == EPI_RESID) {
            const double f = a.f[a.f_shared ? p : o];
            a.out[o] = f - kv;
        } else {   // EPI_CHEB
            const double f = a.f[a.f_shared ? p : o];
            const double dg = g.gv.diag[gi] * g.gh.diag[gj] + l2 * g.S.c[p];
            const double* cc = a.cheb + (size_t)slot * a.cheb_stride;
            const double dn = cc[0] * a.d[o] + cc[1] * (f - kv) / dg;
            a.d[o] = dn;
            a.out[o] = v + dn;
        }
    }
    if (EPI == EPI_DOT) {
        __shared__ double sh[APPLY_THREADS];
        const double s = block_sum<APPLY_THREADS>(dot, sh);
        if (threadIdx.x == 0)
            a.part[(size_t)slot * gridDim.x * gridDim.y + blockIdx.x +
                   (size_t)gridDim.x * blockIdx.y] = s;
    }
}

static size_t apply_lds_bytes(const LevelGeom& g) {
    const int hv = g.gv.bw > 1 ? g.gv.bw : 1, hh = g.gh.bw > 1 ? g.gh.bw : 1;
    const int SY = (TILE_Y + 2 * hv) | 1;
    const int CX = TILE_X + 2 * hh;
    return sizeof(double) * (size_t)CX * (SY + TILE_Y + 1);
}

template <int PRO, int EPI>
static void launch_t(const ApplyArgs& a, hipStream_t s) {
    static bool configured = false;
    if (!configured) {
        // dynamic LDS may use what the kernel's static LDS leaves of 160 KiB
        hipFuncAttributes attr;
        size_t stat = 0;
        if (hipFuncGetAttributes(&attr, (const void*)k_apply<PRO, EPI>) ==
            hipSuccess)
            stat = attr.sharedSizeBytes;
        hipFuncSetAttribute((const void*)k_apply<PRO, EPI>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(160 * 1024 - stat));
        configured = true;
    }
    dim3 grid((a.g.nv + TILE_Y - 1) / TILE_Y, (a.g.nh + TILE_X - 1) / TILE_X,
              a.nslot);
    hipLaunchKernelGGL((k_apply<PRO, EPI>), grid, dim3(APPLY_THREADS),
                       apply_lds_bytes(a.g), s, a);
}

int apply_tiles(const LevelGeom& g) {
    return ((g.nv + TILE_Y - 1) / TILE_Y) * ((g.nh + TILE_X - 1) / TILE_X);
}

void launch_apply(int pro, int epi, const ApplyArgs& a, hipStream_t s) {
    if (pro == PRO_PUPDATE) {
        launch_t<PRO_PUPDATE, EPI_DOT>(a, s);
        return;
    }
    switch (epi) {
        case EPI_STORE: launch_t<PRO_PLAIN, EPI_STORE>(a, s); break;
        case EPI_DOT: launch_t<PRO_PLAIN, EPI_DOT>(a, s); break;
        case EPI_RESID: launch_t<PRO_PLAIN, EPI_RESID>(a, s); break;
        default: launch_t<PRO_PLAIN, EPI_CHEB>(a, s); break;
    }
}

}  // namespace rls
