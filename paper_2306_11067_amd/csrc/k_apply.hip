// Level operator K_k(lambda) v = (G_h (x) G_v) v + lambda^2 S_k v, batched
// over lambda, with a fused prologue (how v is formed while it is loaded)
// and epilogue (what is done with K v).  One workgroup computes one output
// tile of one lambda slot:
//   1. load v on the tile plus a halo into LDS (the Gram band's index map
//      supplies wrap / reflection / zero outside the grid), applying the
//      prologue at every loaded point; stage the band coefficients in LDS;
//   2. vertical pass of G_v for every loaded column;
//   3. horizontal pass of G_h;
//   4. add lambda^2 times the 9-point stencil S_k read from the LDS tile;
//   5. epilogue.
// This is the two-stage level product of the paper's Section 3.2: for the
// blur the products with A_k and A_k^T collapse into the separable Gram
// A_k^T A_k = G_h (x) G_v, and M_k^T M_k is the Galerkin stencil of
// L^T D^2 L.  The prologues and epilogues fuse the surrounding steps of the
// V-cycle (Algorithm 1) and of PCG into the same pass over the tile.
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "pcg_ctl.h"

namespace rls {

__device__ __forceinline__ double diag_at(const LevelGeom& g, double l2,
                                          int i, int j, int64_t p) {
    return g.gv.diag[i] * g.gh.diag[j] + l2 * g.S.c[p];
}

// Coarse points contributing to fine point f and their weights (linear
// interpolation, vertex-centred).
__device__ __forceinline__ int interp_sources(int f, int nf, int periodic,
                                              int* I, double* w) {
    const int nc = nf >> 1;
    if ((f & 1) == 0) { I[0] = f >> 1; w[0] = 1.0; return 1; }
    const int c = f >> 1;
    if (c + 1 < nc) { I[0] = c; I[1] = c + 1; w[0] = w[1] = 0.5; return 2; }
    if (periodic) { I[0] = c; I[1] = 0; w[0] = w[1] = 0.5; return 2; }
    I[0] = c; w[0] = 1.0; return 1;
}

// (P e)(fi, fj) for the coarse vector e of size (nf_v/2) x (nf_h/2).
__device__ __forceinline__ double prolong_at(const double* __restrict__ e,
                                             int fi, int fj, int nvf, int nhf,
                                             int periodic) {
    int Ii[2], Jj[2];
    double wi[2], wj[2];
    const int ni = interp_sources(fi, nvf, periodic, Ii, wi);
    const int nj = interp_sources(fj, nhf, periodic, Jj, wj);
    const int64_t nvc = nvf >> 1;
    double s = 0.0;
    for (int b = 0; b < nj; ++b) {
        double cs = 0.0;
        for (int a = 0; a < ni; ++a) cs += wi[a] * e[Ii[a] + nvc * Jj[b]];
        s += wj[b] * cs;
    }
    return s;
}

// Register window of the vertical pass for uniform bands: each thread
// produces VWIN consecutive rows of one column, consuming the taps VCH at
// a time (taps zero-padded to a multiple of VCH).
constexpr int VWIN = 8;
constexpr int VCH = 8;

struct TileShape {
    int lo, hv, hh, RY, SY, CX, SO, RO, CO, SR, WV, WVP, WH, NCV, NCH;
    __host__ __device__ TileShape(const LevelGeom& g, int ext) {
        lo = ext;
        hv = (g.gv.bw > 1 ? g.gv.bw : 1) + lo;
        hh = (g.gh.bw > 1 ? g.gh.bw : 1) + lo;
        RY = TILE_Y + 2 * hv;
        SY = (RY + VWIN + VCH) | 1;   // slack rows read by the last window
        CX = TILE_X + 2 * hh;
        RO = TILE_Y + lo;             // output rows (incl. low extension)
        CO = TILE_X + lo;
        SO = RO | 1;
        SR = RO | 1;
        WV = 2 * g.gv.bw + 1;
        WVP = (WV + VCH - 1) / VCH * VCH;
        WH = 2 * g.gh.bw + 1;
        NCV = g.gv.uniform ? 1 : RO;  // staged coefficient rows
        NCH = g.gh.uniform ? 1 : CO;
    }
    __host__ __device__ size_t lds_doubles(int restrict_) const {
        return (size_t)CX * SY + (size_t)CX * SO +
               (restrict_ ? (size_t)CO * SR : 0) + (size_t)NCV * WVP +
               (size_t)NCH * WH;
    }
};

// Vertical pass of a uniform band with the chunked register window.
__device__ __forceinline__ void vert_window(const double* __restrict__ vin,
                                            double* __restrict__ vt,
                                            const double* __restrict__ taps,
                                            const TileShape& T, int bw, int i0,
                                            int nv, int per) {
    const int nseg = (T.RO + VWIN - 1) / VWIN;
    for (int e = threadIdx.x; e < nseg * T.CX; e += APPLY_THREADS) {
        const int sg = e / T.CX, jj = e - sg * T.CX;   // lanes along columns
        const int r0 = sg * VWIN;
        const double* col = vin + jj * T.SY + r0 - T.lo + T.hv - bw;
        double acc[VWIN];
#pragma unroll
        for (int o = 0; o < VWIN; ++o) acc[o] = 0.0;
        for (int c0 = 0; c0 < T.WVP; c0 += VCH) {
            double win[VWIN + VCH - 1];
            double tp[VCH];
#pragma unroll
            for (int m = 0; m < VWIN + VCH - 1; ++m) win[m] = col[c0 + m];
#pragma unroll
            for (int k = 0; k < VCH; ++k) tp[k] = taps[c0 + k];
#pragma unroll
            for (int k = 0; k < VCH; ++k)
#pragma unroll
                for (int o = 0; o < VWIN; ++o) acc[o] += tp[k] * win[o + k];
        }
#pragma unroll
        for (int o = 0; o < VWIN; ++o) {
            const int r = r0 + o;
            if (r >= T.RO) break;
            const int gi = i0 + r - T.lo;
            const bool ok = gi < nv && (gi >= 0 || per);
            vt[jj * T.SO + r] = ok ? acc[o] : 0.0;
        }
    }
}

// Per-output operands of the epilogue, loaded from global memory before
// the tile's barriers so that their latency overlaps the tile load.
struct OutPre {
    bool ok;
    int gi, gj;
    double sc, sn, snm, se, sem, sne, snem, sse, ssep;   // stencil couplings
    double f, d, dg;                                    // rhs, direction, diag
};

template <int PRO, int EPI>
__device__ __forceinline__ void out_load(OutPre& q, int e, const ApplyArgs& a,
                                         const TileShape& T, int i0, int j0,
                                         size_t so, double l2) {
    const LevelGeom& g = a.g;
    const int nv = g.nv, nh = g.nh, per = g.S.periodic;
    const int c = e / T.RO, r = e - c * T.RO;
    int gi = i0 + r - T.lo, gj = j0 + c - T.lo;
    q.ok = gi < nv && (gi >= 0 || per) && gj < nh && (gj >= 0 || per);
    if (!q.ok) return;
    if (gi < 0) gi += nv;
    if (gj < 0) gj += nh;
    q.gi = gi;
    q.gj = gj;
    const int64_t p = gi + (int64_t)nv * gj;
    int im = gi - 1, jm = gj - 1, ip = gi + 1;
    const bool okim = wrap_or_drop(im, nv, per);
    const bool okjm = wrap_or_drop(jm, nh, per);
    const bool okip = wrap_or_drop(ip, nv, per);
    q.sc = g.S.c[p];
    q.sn = g.S.cn[p];
    q.snm = okim ? g.S.cn[im + (int64_t)nv * gj] : 0.0;
    q.se = g.S.ce[p];
    q.sem = okjm ? g.S.ce[gi + (int64_t)nv * jm] : 0.0;
    if (g.S.nine) {
        q.sne = g.S.cne[p];
        q.snem = (okim && okjm) ? g.S.cne[im + (int64_t)nv * jm] : 0.0;
        q.sse = g.S.cse[p];
        q.ssep = (okip && okjm) ? g.S.cse[ip + (int64_t)nv * jm] : 0.0;
    }
    const size_t o = so + p;
    if (EPI == EPI_RESID || EPI == EPI_RESTRICT || EPI == EPI_CHEB)
        q.f = a.f[a.f_shared ? p : o];
    if (EPI == EPI_CHEB) {
        q.d = PRO == PRO_JACOBI ? 0.0 : a.d[o];
        q.dg = g.gv.diag[gi] * g.gh.diag[gj] + l2 * q.sc;
    }
}

template <int PRO, int EPI>
__device__ __forceinline__ void apply_body(const ApplyArgs& a, double* lds,
                                           double* red) {
    constexpr int EXT = EPI == EPI_RESTRICT ? 1 : 0;
    const int slot = a.slots ? a.slots[blockIdx.z] : (int)blockIdx.z;
    if (a.active && !a.active[slot]) return;
    const LevelGeom& g = a.g;
    const int nv = g.nv, nh = g.nh;
    const int64_t n = (int64_t)nv * nh;
    // XCD-aware tile order: workgroups are dealt round-robin over the 8
    // XCDs, so give each XCD a contiguous run of tiles (shared halos stay
    // in that XCD's L2) when the tile count allows it.
    const int ntx = gridDim.x, nty = gridDim.y, ntile = ntx * nty;
    int tile = blockIdx.x + ntx * blockIdx.y;
    if ((ntile & 7) == 0) tile = (tile & 7) * (ntile >> 3) + (tile >> 3);
    const int tx = tile % ntx, ty = tile / ntx;
    const int i0 = tx * TILE_Y, j0 = ty * TILE_X;
    const TileShape T(g, EXT);
    const int bwv = g.gv.bw, bwh = g.gh.bw;
    double* vin = lds;
    double* vt = vin + T.CX * T.SY;
    double* rs = vt + T.CX * T.SO;
    double* cv = rs + (EXT ? T.CO * T.SR : 0);
    double* ch = cv + T.NCV * T.WVP;
    const size_t so = (size_t)slot * n;
    const double* src = a.in ? a.in + so : nullptr;
    const double l2 = a.lam2[slot];
    const int per = g.S.periodic;

    // PCG scalars folded into this kernel; tile 0 of a slot leads
    const bool lead = tile == 0;
    double beta = 0.0, cj = 0.0;
    if (PRO == PRO_PUPDATE) {
        if (!pcg_beta<APPLY_THREADS>(a.st, a.active_w, slot, a.part_rz, a.nrz,
                                     a.parity, lead, red, beta))
            return;
    }
    if (a.gate) {
        if (!pcg_gate<APPLY_THREADS>(a.st, a.active_w, slot, a.part_rr, a.nrr,
                                     lead, red))
            return;
    }
    if (PRO == PRO_JACOBI || PRO == PRO_PROLONG_JAC)
        cj = a.cheb_first[(size_t)slot * a.cheb_stride + 1];

    // 0. operands of this thread's first output, in flight during the load
    OutPre pre;
    const int nout = T.RO * T.CO;
    if ((int)threadIdx.x < nout)
        out_load<PRO, EPI>(pre, threadIdx.x, a, T, i0, j0, so, l2);

    // 1. stage band coefficients, load v with prologue
    for (int e = threadIdx.x; e < T.NCV * T.WVP; e += APPLY_THREADS) {
        const int r = e / T.WVP, k = e - r * T.WVP;
        double c = 0.0;
        if (k < T.WV) {                           // zero padding to WVP
            if (g.gv.uniform) {
                c = g.gv.taps[k];
            } else {
                int gi = i0 + r - T.lo;
                if (gi < 0 && per) gi += nv;
                if (gi >= 0 && gi < nv) c = g.gv.table[(size_t)gi * T.WV + k];
            }
        }
        cv[e] = c;
    }
    for (int e = threadIdx.x; e < T.NCH * T.WH; e += APPLY_THREADS) {
        const int c0 = e / T.WH, k = e - c0 * T.WH;
        double c = 0.0;
        if (g.gh.uniform) {
            c = g.gh.taps[k];
        } else {
            int gj = j0 + c0 - T.lo;
            if (gj < 0 && per) gj += nh;
            if (gj >= 0 && gj < nh) c = g.gh.table[(size_t)gj * T.WH + k];
        }
        ch[e] = c;
    }
    for (int e = threadIdx.x; e < T.CX * T.RY; e += APPLY_THREADS) {
        const int jj = e / T.RY, ii = e - jj * T.RY;
        const int ui = i0 - T.hv + ii, uj = j0 - T.hh + jj;
        bool okv, okh;
        const int gi = map_index(ui, nv, g.gv.map, okv);
        const int gj = map_index(uj, nh, g.gh.map, okh);
        double v = 0.0;
        if (okv && okh) {
            const int64_t p = gi + (int64_t)nv * gj;
            if (PRO == PRO_PLAIN) {
                v = src[p];
            } else if (PRO == PRO_PUPDATE) {
                const double po = beta == 0.0 ? 0.0 : a.pold[so + p];
                v = src[p] + beta * po;
                const bool own = ii >= T.hv && ii < T.hv + TILE_Y &&
                                 jj >= T.hh && jj < T.hh + TILE_X && ui < nv &&
                                 uj < nh;
                if (own) a.pnew[so + p] = v;
            } else if (PRO == PRO_JACOBI) {
                v = cj * a.f[a.f_shared ? p : so + p] / diag_at(g, l2, gi, gj, p);
            } else if (PRO == PRO_PROLONG) {
                v = src[p] + prolong_at(a.ec + (size_t)slot * (n >> 2), gi, gj,
                                        nv, nh, per);
            } else {   // PRO_PROLONG_JAC
                v = cj * a.f[a.f_shared ? p : so + p] / diag_at(g, l2, gi, gj, p) +
                    prolong_at(a.ec + (size_t)slot * (n >> 2), gi, gj, nv, nh, per);
            }
        }
        vin[jj * T.SY + ii] = v;
    }
    __syncthreads();

    // 2. vertical pass over output rows [-lo, TILE_Y) of every loaded column
    if (g.gv.uniform) {
        vert_window(vin, vt, cv, T, bwv, i0, nv, per);
    } else
    for (int e = threadIdx.x; e < T.RO * T.CX; e += APPLY_THREADS) {
        const int jj = e / T.RO, r = e - jj * T.RO;        // r = row + lo
        const int gi = i0 + r - T.lo;
        double s = 0.0;
        if (gi < nv && (gi >= 0 || per)) {
            const double* col = vin + jj * T.SY + r - T.lo + T.hv - bwv;
            const double* cf = cv + r * T.WVP;
#pragma unroll 4
            for (int k = 0; k < T.WV; ++k) s += cf[k] * col[k];
        }
        vt[jj * T.SO + r] = s;
    }
    __syncthreads();

    // 3.-5. horizontal pass, stencil, epilogue
    double dot = 0.0;
    for (int e = threadIdx.x; e < nout; e += APPLY_THREADS) {
        const int c = e / T.RO, r = e - c * T.RO;          // local + lo
        OutPre q;
        if (e == (int)threadIdx.x) q = pre;
        else out_load<PRO, EPI>(q, e, a, T, i0, j0, so, l2);
        if (!q.ok) {
            if (EXT) rs[c * T.SR + r] = 0.0;
            continue;
        }
        double kv = 0.0;
        {
            const double* row = vt + (c - T.lo + T.hh - bwh) * T.SO + r;
            const double* cf = ch + (g.gh.uniform ? 0 : c) * T.WH;
#pragma unroll 4
            for (int k = 0; k < T.WH; ++k) kv += cf[k] * row[k * T.SO];
        }
        const double* vc = vin + (c - T.lo + T.hh) * T.SY + r - T.lo + T.hv;
        double sv = q.sc * vc[0];
        sv += q.sn * vc[1];
        sv += q.snm * vc[-1];
        sv += q.se * vc[T.SY];
        sv += q.sem * vc[-T.SY];
        if (g.S.nine) {
            sv += q.sne * vc[T.SY + 1];
            sv += q.snem * vc[-T.SY - 1];
            sv += q.sse * vc[T.SY - 1];
            sv += q.ssep * vc[-T.SY + 1];
        }
        kv += l2 * sv;
        const double v = vc[0];
        const size_t o = so + q.gi + (int64_t)nv * q.gj;
        if (EPI == EPI_STORE) {
            a.out[o] = kv;
        } else if (EPI == EPI_DOT) {
            a.out[o] = kv;
            dot += v * kv;
        } else if (EPI == EPI_RESID) {
            a.out[o] = q.f - kv;
        } else if (EPI == EPI_RESTRICT) {
            rs[c * T.SR + r] = q.f - kv;
        } else {   // EPI_CHEB
            const double* cc = a.cheb + (size_t)slot * a.cheb_stride;
            const double dprev = PRO == PRO_JACOBI ? v : q.d;
            const double dn = cc[0] * dprev + cc[1] * (q.f - kv) / q.dg;
            a.d[o] = dn;
            const double xn = v + dn;
            a.out[o] = xn;
            if (a.dot) dot += q.f * xn;
        }
    }
    if (EPI == EPI_RESTRICT) {
        // full weighting of the residual tile onto the coarse points whose
        // centre lies in the tile: fc(I, J) = sum P(f, (I, J)) res(f)
        __syncthreads();
        const int nvc = nv >> 1, nhc = nh >> 1;
        const int I0 = i0 >> 1, J0 = j0 >> 1;
        constexpr int CI = TILE_Y / 2, CJ = TILE_X / 2;
        for (int e = threadIdx.x; e < CI * CJ; e += APPLY_THREADS) {
            const int cjj = e / CI, cii = e - cjj * CI;
            const int I = I0 + cii, J = J0 + cjj;
            if (I >= nvc || J >= nhc) continue;
            double s = 0.0;
            for (int b = -1; b <= 1; ++b) {
                int fj = 2 * J + b;
                if (!wrap_or_drop(fj, nh, per)) continue;
                const double wj = interp_weight(fj, J, nh, per);
                if (wj == 0.0) continue;
                const int lc = 2 * cjj + b + 1;             // local column + lo
                double cs = 0.0;
                for (int a2 = -1; a2 <= 1; ++a2) {
                    int fi = 2 * I + a2;
                    if (!wrap_or_drop(fi, nv, per)) continue;
                    const double wi = interp_weight(fi, I, nv, per);
                    if (wi != 0.0) cs += wi * rs[lc * T.SR + 2 * cii + a2 + 1];
                }
                s += wj * cs;
            }
            a.fc[(size_t)slot * nvc * nhc + I + (int64_t)nvc * J] = s;
        }
    }
    if (EPI == EPI_DOT || (EPI == EPI_CHEB && a.dot)) {
        const double s = block_sum<APPLY_THREADS>(dot, red);
        if (threadIdx.x == 0)
            a.part[(size_t)slot * a.part_stride + tile] = s;
    }
}

template <int PRO, int EPI>
__global__ void __launch_bounds__(APPLY_THREADS) k_apply(ApplyArgs a) {
    extern __shared__ double lds[];
    __shared__ double red[APPLY_THREADS];
    apply_body<PRO, EPI>(a, lds, red);
}

// The finest-level Chebyshev step (plain prologue) under a name of its own,
// so that profiles separate the sweep's most frequent kernel from the same
// step on coarser levels.
__global__ void __launch_bounds__(APPLY_THREADS) k_smooth_fine(ApplyArgs a) {
    extern __shared__ double lds[];
    __shared__ double red[APPLY_THREADS];
    apply_body<PRO_PLAIN, EPI_CHEB>(a, lds, red);
}

template <int PRO, int EPI>
static void configure_one() {
    // dynamic LDS may use what the kernel's static LDS leaves of 160 KiB
    hipFuncAttributes attr;
    size_t stat = 0;
    if (hipFuncGetAttributes(&attr, (const void*)k_apply<PRO, EPI>) == hipSuccess)
        stat = attr.sharedSizeBytes;
    (void)hipFuncSetAttribute((const void*)k_apply<PRO, EPI>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(160 * 1024 - stat));
}

template <int PRO, int EPI>
static void launch_one(const ApplyArgs& a, hipStream_t s) {
    const TileShape T(a.g, EPI == EPI_RESTRICT);
    dim3 grid((a.g.nv + TILE_Y - 1) / TILE_Y, (a.g.nh + TILE_X - 1) / TILE_X,
              a.nslot);
    hipLaunchKernelGGL((k_apply<PRO, EPI>), grid, dim3(APPLY_THREADS),
                       sizeof(double) * T.lds_doubles(EPI == EPI_RESTRICT), s,
                       a);
}

// Every (prologue, epilogue) pair in use.
#define RLS_APPLY_VARIANTS(X)         \
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

void configure_apply_kernels() {
    static bool done = false;
    if (done) return;
#define RLS_CFG(P, E) configure_one<P, E>();
    RLS_APPLY_VARIANTS(RLS_CFG)
#undef RLS_CFG
    {
        hipFuncAttributes attr;
        size_t stat = 0;
        if (hipFuncGetAttributes(&attr, (const void*)k_smooth_fine) == hipSuccess)
            stat = attr.sharedSizeBytes;
        (void)hipFuncSetAttribute((const void*)k_smooth_fine,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(160 * 1024 - stat));
    }
    (void)hipGetLastError();
    done = true;
}

int apply_tiles(const LevelGeom& g) {
    return ((g.nv + TILE_Y - 1) / TILE_Y) * ((g.nh + TILE_X - 1) / TILE_X);
}

size_t apply_lds_bytes(const LevelGeom& g, int epi) {
    const TileShape T(g, epi == EPI_RESTRICT);
    return sizeof(double) * T.lds_doubles(epi == EPI_RESTRICT);
}

void launch_smooth_fine(const ApplyArgs& a, hipStream_t s) {
    const TileShape T(a.g, 0);
    dim3 grid((a.g.nv + TILE_Y - 1) / TILE_Y, (a.g.nh + TILE_X - 1) / TILE_X,
              a.nslot);
    hipLaunchKernelGGL(k_smooth_fine, grid, dim3(APPLY_THREADS),
                       sizeof(double) * T.lds_doubles(0), s, a);
}

void launch_apply(int pro, int epi, const ApplyArgs& a, hipStream_t s) {
#define RLS_LAUNCH(P, E) \
    if (pro == P && epi == E) { launch_one<P, E>(a, s); return; }
    RLS_APPLY_VARIANTS(RLS_LAUNCH)
#undef RLS_LAUNCH
    std::fprintf(stderr, "rls: no level-operator kernel for prologue %d, "
                         "epilogue %d\n", pro, epi);
    std::abort();
}

}  // namespace rls
