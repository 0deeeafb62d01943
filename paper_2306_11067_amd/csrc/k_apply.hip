// Level operator K_k(lambda) v = (G_h (x) G_v) v + lambda^2 S_k v, batched
// over lambda, with a fused prologue (how v is formed while it is loaded)
// and epilogue (what is done with K v).  One 256-thread workgroup computes
// one 64 x 16 output tile of one lambda slot (about 50 KB of LDS, so three
// workgroups share a CU and one's loads overlap another's arithmetic):
//   0. issue the global loads of the per-output operands (right-hand side,
//      direction, stencil couplings);
//   1. load v on the tile plus a halo into LDS (the Gram band's index map
//      supplies wrap / reflection / zero outside the grid), applying the
//      prologue at every loaded point; stage the band coefficients;
//   2. horizontal pass of G_h over the output columns and the extended
//      rows (register windows of 8 columns);
//   3. vertical pass of G_v over the output rows (windows of 8 rows);
//   4. add lambda^2 times the 9-point stencil S_k read from the LDS tile and
//      apply the epilogue, lanes along the contiguous axis.
// The horizontal pass runs first because the tile is taller than wide: the
// first pass is evaluated on the halo of the second, 92 rows for 64 here.
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

// Element idx of an array with a workgroup-uniform base: a 32-bit byte
// offset on a scalar base (grids are limited to 2^28 points per slot).
template <class R>
__device__ __forceinline__ R ldu(const R* base, uint32_t idx) {
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base) +
                                       idx * (uint32_t)sizeof(R));
}
template <class R>
__device__ __forceinline__ void stu(R* base, uint32_t idx, R v) {
    *reinterpret_cast<R*>(reinterpret_cast<char*>(base) +
                          idx * (uint32_t)sizeof(R)) = v;
}
// Vector element in the arithmetic type R, stored as V.
template <class R, class V>
__device__ __forceinline__ R ldv(const V* base, uint32_t idx) {
    return Cvt<R, V>::in(ldu(base, idx));
}
template <class R, class V>
__device__ __forceinline__ void stv(V* base, uint32_t idx, R v) {
    stu(base, idx, Cvt<R, V>::out(v));
}

template <class R>
__device__ __forceinline__ R diag_at(const LevelGeomT<R>& g, R l2, int i,
                                     int j, uint32_t p) {
    return g.gv.diag[i] * g.gh.diag[j] + l2 * ldu(g.S.c, p);
}

// Coarse points contributing to fine point f and their weights (linear
// interpolation, vertex-centred).
template <class R>
__device__ __forceinline__ int interp_sources(int f, int nf, int periodic,
                                              int* I, R* w) {
    const int nc = nf >> 1;
    if ((f & 1) == 0) { I[0] = f >> 1; w[0] = R(1); return 1; }
    const int c = f >> 1;
    if (c + 1 < nc) { I[0] = c; I[1] = c + 1; w[0] = w[1] = R(0.5); return 2; }
    if (periodic) { I[0] = c; I[1] = 0; w[0] = w[1] = R(0.5); return 2; }
    I[0] = c; w[0] = R(1); return 1;
}

// (P e)(fi, fj) for the coarse vector e of size (nf_v/2) x (nf_h/2).
template <class R, class V>
__device__ __forceinline__ R prolong_at(const V* __restrict__ e, int fi,
                                        int fj, int nvf, int nhf,
                                        int periodic) {
    int Ii[2], Jj[2];
    R wi[2], wj[2];
    const int ni = interp_sources(fi, nvf, periodic, Ii, wi);
    const int nj = interp_sources(fj, nhf, periodic, Jj, wj);
    const int64_t nvc = nvf >> 1;
    R s = R(0);
    for (int b = 0; b < nj; ++b) {
        R cs = R(0);
        for (int a = 0; a < ni; ++a)
            cs += wi[a] * Cvt<R, V>::in(e[Ii[a] + nvc * Jj[b]]);
        s += wj[b] * cs;
    }
    return s;
}

// Register windows of the two band passes: a thread produces HWIN (VWIN)
// consecutive outputs of one row (column), consuming the taps CH at a time.
// Tap lists are zero-padded to a multiple of CH, and the LDS lines the
// padded taps reach are zero-filled, so no undefined value enters a sum.
constexpr int HWIN = 8;
constexpr int VWIN = 8;
constexpr int CH = 8;
// outputs whose operands a thread loads before the tile (every tile has at
// least TILE_Y * TILE_X outputs)
constexpr int NPRE = TILE_Y * TILE_X / APPLY_THREADS;
static_assert(NPRE * APPLY_THREADS == TILE_Y * TILE_X, "tile / block mismatch");
static_assert((TILE_X + 1) * ((TILE_Y + VWIN) / VWIN) <= APPLY_THREADS,
              "one vertical window per thread");

__host__ __device__ constexpr int round_up(int x, int m) {
    return (x + m - 1) / m * m;
}

// Geometry of one tile.  Output point (r, c), r in [0, RO), c in [0, CO),
// is grid point (i0 + r - lo, j0 + c - lo); lo = 1 adds the low row and
// column the full-weighting restriction needs.  The input tile holds v on
// rows ii in [0, RY) <-> i0 - hv + ii and columns jj in [0, CX) <->
// j0 - hh + jj, row-major with row stride SX (odd: conflict-free when
// lanes run along rows).
struct TileShape {
    int lo, bwv, bwh, hv, hh;
    int RY, CX, SX;         // input rows, columns, row stride (>= CX)
    int RO, CO;             // output rows / columns
    int NWH, NWV;           // windows per output row / column
    int NHR, SH;            // rows of the horizontal-pass result, stride
    int SR;                 // column stride of the staged K v
    int WV, WVP, WH, WHP;   // tap counts, padded to CH
    int NCV, NCH;           // staged coefficient lines (1: uniform band)
    template <class R>
    __host__ __device__ TileShape(const LevelGeomT<R>& g, int ext) {
        lo = ext;
        bwv = g.gv.bw;
        bwh = g.gh.bw;
        hv = (bwv > 1 ? bwv : 1) + lo;
        hh = (bwh > 1 ? bwh : 1) + lo;
        RY = TILE_Y + 2 * hv;
        CX = TILE_X + 2 * hh;
        RO = TILE_Y + lo;
        CO = TILE_X + lo;
        WV = 2 * bwv + 1;
        WVP = round_up(WV, CH);
        WH = 2 * bwh + 1;
        WHP = round_up(WH, CH);
        NWH = (CO + HWIN - 1) / HWIN;
        NWV = (RO + VWIN - 1) / VWIN;
        // one past the last input column a horizontal window reads
        const int cend = NWH * HWIN + WHP - 1 - lo + hh - bwh;
        SX = (cend > CX ? cend : CX) | 1;
        NHR = RO + 2 * bwv;
        SH = (NWV * VWIN + WVP - 1) | 1;
        SR = RO | 1;
        NCV = g.gv.uniform ? 1 : NWV * VWIN;
        NCH = g.gh.uniform ? 1 : NWH * HWIN;
    }
    // the horizontal-pass result, reused for K v (and the residual)
    __host__ __device__ size_t ht_elems() const {
        const size_t x = (size_t)CO * SH, y = (size_t)CO * SR;
        return x > y ? x : y;
    }
    // LDS elements (of the level's value type)
    __host__ __device__ size_t lds_elems() const {
        return (size_t)RY * SX + ht_elems() + (size_t)NCV * WVP +
               (size_t)NCH * WHP + RO + CO;
    }
};

// Grid point of output e, false outside the grid.
template <class R>
__device__ __forceinline__ bool out_index(int e, const TileShape& T,
                                          const LevelGeomT<R>& g, int i0, int j0,
                                          int& gi, int& gj) {
    const int nv = g.nv, nh = g.nh, per = g.S.periodic;
    const int c = e / T.RO, r = e - c * T.RO;
    gi = i0 + r - T.lo;
    gj = j0 + c - T.lo;
    if (!(gi < nv && (gi >= 0 || per) && gj < nh && (gj >= 0 || per)))
        return false;
    if (gi < 0) gi += nv;
    if (gj < 0) gj += nh;
    return true;
}

// The slot's arrays (uniform over the workgroup), V the storage type.
template <class V>
struct SlotPtrs {
    const V* src;   // operand v (or z for the p update)
    const V* pold;  // previous search direction
    const V* f;     // right-hand side
    V* d;           // Chebyshev direction
    V* out;         // result
    V* pnew;        // new search direction
};

// Operands of one output point from global memory, requested before the
// tile load so that they arrive with it: right-hand side and Chebyshev
// direction (per lambda) and the five-point part of the stencil (centre,
// north, south, east, west couplings; zero across a non-periodic edge).
template <class R>
struct OutPre {
    R f, d, sc, sn, ss, se, sw;
};

template <int PRO, int EPI, class R, class V>
__device__ __forceinline__ void out_load(OutPre<R>& q, int e,
                                         const ApplyArgsT<R, V>& a,
                                         const SlotPtrs<V>& sp,
                                         const TileShape& T, int i0, int j0) {
    const LevelGeomT<R>& g = a.g;
    const int nv = g.nv, nh = g.nh, per = g.S.periodic;
    q.f = q.d = q.sc = q.sn = q.ss = q.se = q.sw = R(0);
    int gi, gj;
    if (!out_index(e, T, g, i0, j0, gi, gj)) return;
    const uint32_t p = gi + (uint32_t)nv * gj;
    int im = gi - 1, jm = gj - 1;
    const bool okim = wrap_or_drop(im, nv, per);
    const bool okjm = wrap_or_drop(jm, nh, per);
    q.sc = ldu(g.S.c, p);
    q.sn = ldu(g.S.cn, p);
    if (okim) q.ss = ldu(g.S.cn, im + (uint32_t)nv * gj);
    q.se = ldu(g.S.ce, p);
    if (okjm) q.sw = ldu(g.S.ce, gi + (uint32_t)nv * jm);
    if (EPI == EPI_RESID || EPI == EPI_RESTRICT || EPI == EPI_CHEB)
        q.f = ldv<R>(sp.f, p);
    if (EPI == EPI_CHEB && PRO != PRO_JACOBI) q.d = ldv<R>(sp.d, p);
}

// Stencil term and epilogue at output e; K v's Gram part is staged in kvs.
template <int PRO, int EPI, class R, class V>
__device__ __forceinline__ void out_point(const OutPre<R>& q, int e,
                                          const ApplyArgsT<R, V>& a,
                                          const SlotPtrs<V>& sp,
                                          const TileShape& T, const R* vin,
                                          R* kvs, R l2, const R* dgl, R c0,
                                          R c1, int i0, int j0, double& dot) {
    const int c = e / T.RO, r = e - c * T.RO;
    const LevelGeomT<R>& g = a.g;
    int gi, gj;
    if (!out_index(e, T, g, i0, j0, gi, gj)) {
        if (EPI == EPI_RESTRICT) kvs[c * T.SR + r] = R(0);
        return;
    }
    const int nv = g.nv, nh = g.nh, per = g.S.periodic;
    const uint32_t p = gi + (uint32_t)nv * gj;
    const R* vc = vin + (r - T.lo + T.hv) * T.SX + c - T.lo + T.hh;
    R sv = q.sc * vc[0];
    sv += q.sn * vc[T.SX];
    sv += q.ss * vc[-T.SX];
    sv += q.se * vc[1];
    sv += q.sw * vc[-1];
    if (g.S.nine) {
        int im = gi - 1, jm = gj - 1, ip = gi + 1;
        const bool okim = wrap_or_drop(im, nv, per);
        const bool okjm = wrap_or_drop(jm, nh, per);
        const bool okip = wrap_or_drop(ip, nv, per);
        sv += ldu(g.S.cne, p) * vc[T.SX + 1];
        if (okim && okjm) sv += ldu(g.S.cne, im + (uint32_t)nv * jm) * vc[-T.SX - 1];
        sv += ldu(g.S.cse, p) * vc[-T.SX + 1];
        if (okip && okjm) sv += ldu(g.S.cse, ip + (uint32_t)nv * jm) * vc[T.SX - 1];
    }
    const R kv = kvs[c * T.SR + r] + l2 * sv;
    const R v = vc[0];
    if (EPI == EPI_STORE) {
        stv(sp.out, p, kv);
    } else if (EPI == EPI_DOT) {
        stv(sp.out, p, kv);
        dot += (double)v * (double)kv;
    } else if (EPI == EPI_RESID) {
        stv(sp.out, p, q.f - kv);
    } else if (EPI == EPI_RESTRICT) {
        kvs[c * T.SR + r] = q.f - kv;
    } else {   // EPI_CHEB
        const R dg = dgl[r] * dgl[T.RO + c] + l2 * q.sc;
        const R dprev = PRO == PRO_JACOBI ? v : q.d;
        const R dn = c0 * dprev + c1 * (q.f - kv) / dg;
        stv(sp.d, p, dn);
        const R xn = v + dn;
        stv(sp.out, p, xn);
        if (a.dot) dot += (double)q.f * (double)xn;
    }
}

template <int PRO, int EPI, class R, class V>
__device__ __forceinline__ void apply_body(const ApplyArgsT<R, V>& a, R* lds,
                                           double* red) {
    constexpr int EXT = EPI == EPI_RESTRICT ? 1 : 0;
    constexpr int NT = APPLY_THREADS;
    const int t = threadIdx.x;
    const int z = blockIdx.z;
    const int slot = z < a.zn ? a.zslot[z] : a.slots ? a.slots[z] : z;
    // A slot that stopped inside a replayed chunk is skipped.  Variants
    // without folded PCG scalars only test the flag once their loads are
    // in flight (reading a stopped slot is harmless, writing is not).
    const bool act = !a.active || a.active[slot];
    constexpr bool SCALARS = PRO == PRO_PUPDATE;
    if ((SCALARS || a.gate) && !act) return;
    const LevelGeomT<R>& g = a.g;
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
    R* vin = lds;
    R* ht = vin + (size_t)T.RY * T.SX;
    R* kvs = ht;                      // after the vertical pass
    R* cv = ht + T.ht_elems();
    R* ch = cv + (size_t)T.NCV * T.WVP;
    R* dgl = ch + (size_t)T.NCH * T.WHP;   // diag G_v rows, diag G_h cols
    const size_t so = (size_t)slot * n;
    SlotPtrs<V> sp;
    sp.src = a.in ? a.in + so : nullptr;
    sp.pold = a.pold ? a.pold + so : nullptr;
    sp.f = a.f ? (a.f_shared ? a.f : a.f + so) : nullptr;
    sp.d = a.d ? a.d + so : nullptr;
    sp.out = a.out ? a.out + so : nullptr;
    sp.pnew = a.pnew ? a.pnew + so : nullptr;
    const R l2 = (R)a.lam2[slot];
    const int per = g.S.periodic;

    // PCG scalars folded into this kernel; tile 0 of a slot leads
    const bool lead = tile == 0;
    double beta = 0.0;
    R cj = R(0);
    if (PRO == PRO_PUPDATE) {
        if (!pcg_beta<NT>(a.st, a.active_w, slot, a.part_rz, a.nrz, a.parity,
                          a.flex ? a.part_zq : nullptr, lead, red, beta))
            return;
    }
    if (a.gate) {
        if (!pcg_gate<NT>(a.st, a.active_w, slot, a.part_rr, a.nrr, lead, red))
            return;
    }
    if (PRO == PRO_JACOBI || PRO == PRO_PROLONG_JAC)
        cj = (R)a.cheb_first[(size_t)slot * a.cheb_stride + 1];
    R c0 = R(0), c1 = R(0);
    if (EPI == EPI_CHEB) {
        c0 = (R)a.cheb[(size_t)slot * a.cheb_stride];
        c1 = (R)a.cheb[(size_t)slot * a.cheb_stride + 1];
    }

    // 1. everything the tile needs from global memory is requested before
    //    the first LDS write: uniform taps (one per thread), v on the tile
    //    plus halo with the prologue applied (batches of LB loads per
    //    thread, no store in between), and the per-output operands of the
    //    epilogue, which stay in flight through the band passes.
    R tapv = R(0), taph = R(0), dgt = R(0);
    if (g.gv.uniform && t < T.WV) tapv = g.gv.taps[t];
    if (g.gh.uniform && t < T.WH) taph = g.gh.taps[t];
    if (EPI == EPI_CHEB && t < T.RO + T.CO) {
        // diagonal of G_v at output row t, of G_h at output column t - RO
        const bool row = t < T.RO;
        const int nn = row ? nv : nh;
        int gx = row ? i0 + t - T.lo : j0 + (t - T.RO) - T.lo;
        if (gx < 0 && per) gx += nn;
        if (gx >= 0 && gx < nn) dgt = row ? g.gv.diag[gx] : g.gh.diag[gx];
    }
    // Each thread keeps one tile row (lanes along the contiguous axis, the
    // row's index map evaluated once) and walks every second column; the
    // loads of a batch of LB columns are issued back to back.
    constexpr int RL = APPLY_THREADS / 2;
    constexpr int LB = PRO == PRO_PLAIN || PRO == PRO_PUPDATE ? 24
                       : PRO == PRO_JACOBI                      ? 12
                                                                : 6;
    OutPre<R> pre[NPRE];
    const int il = t & (RL - 1), jl = t / RL;
    for (int rb = 0; rb < T.RY; rb += RL) {
        const int ii = rb + il;
        const bool rin = ii < T.RY;
        const int ui = i0 - T.hv + ii;
        bool okv;
        const int gi = map_index(ui, nv, g.gv.map, okv);
        for (int cb = 0; cb < T.CX; cb += 2 * LB) {
            R v[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int jj = cb + jl + 2 * u;
                v[u] = R(0);
                bool okh;
                const int gj = map_index(j0 - T.hh + jj, nh, g.gh.map, okh);
                if (rin && okv && jj < T.CX && okh) {
                    const uint32_t p = gi + (uint32_t)nv * gj;
                    if (PRO == PRO_PLAIN) {
                        v[u] = ldv<R>(sp.src, p);
                    } else if (PRO == PRO_PUPDATE) {
                        // p_old is undefined before the first iteration
                        const R po = beta == 0.0 ? R(0) : ldv<R>(sp.pold, p);
                        v[u] = ldv<R>(sp.src, p) + (R)beta * po;
                    } else if (PRO == PRO_JACOBI) {
                        v[u] = cj * ldv<R>(sp.f, p) / diag_at(g, l2, gi, gj, p);
                    } else if (PRO == PRO_PROLONG) {
                        v[u] = ldv<R>(sp.src, p) +
                               prolong_at<R>(a.ec + (size_t)slot * (n >> 2), gi,
                                             gj, nv, nh, per);
                    } else {   // PRO_PROLONG_JAC
                        v[u] = cj * ldv<R>(sp.f, p) / diag_at(g, l2, gi, gj, p) +
                               prolong_at<R>(a.ec + (size_t)slot * (n >> 2), gi,
                                             gj, nv, nh, per);
                    }
                }
            }
            if (rb == 0 && cb == 0) {
#pragma unroll
                for (int k = 0; k < NPRE; ++k)
                    out_load<PRO, EPI, R, V>(pre[k], t + k * NT, a, sp, T, i0, j0);
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int jj = cb + jl + 2 * u;
                if (rin && jj < T.CX) {
                    vin[ii * T.SX + jj] = v[u];
                    if (PRO == PRO_PUPDATE) {
                        // p_new on the tile's own points
                        const int uj = j0 - T.hh + jj;
                        const bool own = ii >= T.hv && ii < T.hv + TILE_Y &&
                                         jj >= T.hh && jj < T.hh + TILE_X &&
                                         ui < nv && uj < nh;
                        if (own) stv(sp.pnew, ui + (uint32_t)nv * uj, v[u]);
                    }
                }
            }
        }
    }

    if (!SCALARS && !a.gate && !act) return;
    if (EPI == EPI_CHEB && t < T.RO + T.CO) dgl[t] = dgt;

    // band coefficients (zero-padded to a multiple of CH), zero padding of
    // the LDS lines the padded taps reach
    if (g.gv.uniform) {
        if (t < T.WVP) cv[t] = tapv;
    } else {
        for (int e = t; e < T.NCV * T.WVP; e += NT) {
            const int r = e / T.WVP, k = e - r * T.WVP;
            int gi = i0 + r - T.lo;
            if (gi < 0 && per) gi += nv;
            R c = R(0);
            if (k < T.WV && r < T.RO && gi >= 0 && gi < nv)
                c = g.gv.table[(size_t)gi * T.WV + k];
            cv[e] = c;
        }
    }
    if (g.gh.uniform) {
        if (t < T.WHP) ch[t] = taph;
    } else {
        for (int e = t; e < T.NCH * T.WHP; e += NT) {
            const int c0 = e / T.WHP, k = e - c0 * T.WHP;
            int gj = j0 + c0 - T.lo;
            if (gj < 0 && per) gj += nh;
            R c = R(0);
            if (k < T.WH && c0 < T.CO && gj >= 0 && gj < nh)
                c = g.gh.table[(size_t)gj * T.WH + k];
            ch[e] = c;
        }
    }
    {
        const int pad = T.SX - T.CX;
        for (int e = t; e < T.RY * pad; e += NT) {
            const int ii = e / pad;
            vin[ii * T.SX + T.CX + (e - ii * pad)] = R(0);
        }
    }
    {
        const int pad = T.SH - T.NHR;
        for (int e = t; e < T.CO * pad; e += NT) {
            const int c = e / pad, q = T.NHR + (e - c * pad);
            ht[c * T.SH + q] = R(0);
        }
    }
    __syncthreads();

    // 2. horizontal pass of G_h over the rows the vertical pass needs:
    //    ht(q, c) = sum_k G_h(c, k) v(q + hv - lo - bwv, c - lo + hh - bwh + k)
    for (int e = t; e < T.NHR * T.NWH; e += NT) {
        const int w = e / T.NHR, q = e - w * T.NHR;       // lanes along rows
        const int c0 = w * HWIN;
        const R* rowp = vin + (q + T.hv - T.lo - T.bwv) * T.SX +
                             (c0 - T.lo + T.hh - T.bwh);
        R acc[HWIN];
#pragma unroll
        for (int o = 0; o < HWIN; ++o) acc[o] = R(0);
        if (g.gh.uniform) {
            for (int k0 = 0; k0 < T.WHP; k0 += CH) {
                R win[HWIN + CH - 1];
#pragma unroll
                for (int m = 0; m < HWIN + CH - 1; ++m)
                    win[m] = rowp[k0 + m];
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const R tp = ch[k0 + k];
#pragma unroll
                    for (int o = 0; o < HWIN; ++o) acc[o] += tp * win[o + k];
                }
            }
        } else {
            // per-column coefficients: rotating window, one tap at a time
            R win[HWIN];
#pragma unroll
            for (int m = 0; m < HWIN; ++m) win[m] = rowp[m];
            const R* cf = ch + c0 * T.WHP;
            for (int k = 0; k < T.WH; ++k) {
#pragma unroll
                for (int o = 0; o < HWIN; ++o) acc[o] += cf[o * T.WHP + k] * win[o];
#pragma unroll
                for (int o = 0; o < HWIN - 1; ++o) win[o] = win[o + 1];
                win[HWIN - 1] = rowp[k + HWIN];
            }
        }
#pragma unroll
        for (int o = 0; o < HWIN; ++o)
            if (c0 + o < T.CO) ht[(c0 + o) * T.SH + q] = acc[o];
    }
    __syncthreads();

    // 3. vertical pass of G_v: (G v)(r, c) = sum_k G_v(r, k) ht(r + k, c)
    R vacc[VWIN];
    const int vw = t / T.CO, vcol = t - vw * T.CO;        // lanes along columns
    const bool vown = t < T.CO * T.NWV;
    if (vown) {
        const int r0 = vw * VWIN;
        const R* colp = ht + vcol * T.SH + r0;
#pragma unroll
        for (int o = 0; o < VWIN; ++o) vacc[o] = R(0);
        if (g.gv.uniform) {
            for (int k0 = 0; k0 < T.WVP; k0 += CH) {
                R win[VWIN + CH - 1];
#pragma unroll
                for (int m = 0; m < VWIN + CH - 1; ++m) win[m] = colp[k0 + m];
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const R tp = cv[k0 + k];
#pragma unroll
                    for (int o = 0; o < VWIN; ++o) vacc[o] += tp * win[o + k];
                }
            }
        } else {
            R win[VWIN];
#pragma unroll
            for (int m = 0; m < VWIN; ++m) win[m] = colp[m];
            const R* cf = cv + r0 * T.WVP;
            for (int k = 0; k < T.WV; ++k) {
#pragma unroll
                for (int o = 0; o < VWIN; ++o) vacc[o] += cf[o * T.WVP + k] * win[o];
#pragma unroll
                for (int o = 0; o < VWIN - 1; ++o) win[o] = win[o + 1];
                win[VWIN - 1] = colp[k + VWIN];
            }
        }
    }
    __syncthreads();
    if (vown) {
#pragma unroll
        for (int o = 0; o < VWIN; ++o) {
            const int r = vw * VWIN + o;
            if (r < T.RO) kvs[vcol * T.SR + r] = vacc[o];
        }
    }
    __syncthreads();

    // 4. stencil term and epilogue (lanes along the contiguous axis)
    double dot = 0.0;
    const int nout = T.RO * T.CO;
#pragma unroll
    for (int k = 0; k < NPRE; ++k)
        out_point<PRO, EPI, R, V>(pre[k], t + k * NT, a, sp, T, vin, kvs, l2,
                                  dgl, c0, c1, i0, j0, dot);
    for (int e = t + NPRE * NT; e < nout; e += NT) {
        OutPre<R> q;
        out_load<PRO, EPI, R, V>(q, e, a, sp, T, i0, j0);
        out_point<PRO, EPI, R, V>(q, e, a, sp, T, vin, kvs, l2, dgl, c0, c1, i0,
                                  j0, dot);
    }

    if (EPI == EPI_RESTRICT) {
        // full weighting of the residual tile onto the coarse points whose
        // centre lies in the tile: fc(I, J) = sum P(f, (I, J)) res(f)
        __syncthreads();
        const R* rs = kvs;
        const int nvc = nv >> 1, nhc = nh >> 1;
        const int I0 = i0 >> 1, J0 = j0 >> 1;
        constexpr int CI = TILE_Y / 2, CJ = TILE_X / 2;
        for (int e = t; e < CI * CJ; e += NT) {
            const int cjj = e / CI, cii = e - cjj * CI;
            const int I = I0 + cii, J = J0 + cjj;
            if (I >= nvc || J >= nhc) continue;
            R s = R(0);
            for (int b = -1; b <= 1; ++b) {
                int fj = 2 * J + b;
                if (!wrap_or_drop(fj, nh, per)) continue;
                const R wj = (R)interp_weight(fj, J, nh, per);
                if (wj == R(0)) continue;
                const int lc = 2 * cjj + b + 1;             // local column + lo
                R cs = R(0);
                for (int a2 = -1; a2 <= 1; ++a2) {
                    int fi = 2 * I + a2;
                    if (!wrap_or_drop(fi, nv, per)) continue;
                    const R wi = (R)interp_weight(fi, I, nv, per);
                    if (wi != R(0)) cs += wi * rs[lc * T.SR + 2 * cii + a2 + 1];
                }
                s += wj * cs;
            }
            a.fc[(size_t)slot * nvc * nhc + I + (int64_t)nvc * J] =
                Cvt<R, V>::out(s);
        }
    }
    if (EPI == EPI_DOT || (EPI == EPI_CHEB && a.dot)) {
        const double s = block_sum<NT>(dot, red);
        if (t == 0) a.part[(size_t)slot * a.part_stride + tile] = s;
    }
}

// Register budget: RLS_APPLY_WAVES waves per SIMD, i.e. that many
// 256-thread workgroups per CU (2: at most 256 VGPRs).
#ifndef RLS_APPLY_WAVES
#define RLS_APPLY_WAVES 2
#endif
#define RLS_APPLY_BOUNDS           \
    __launch_bounds__(APPLY_THREADS) \
    __attribute__((amdgpu_waves_per_eu(RLS_APPLY_WAVES)))
// FP32 tiles use fewer registers: three workgroups per CU (<= 168 VGPRs).
#define RLS_APPLY_BOUNDS_T(R)      \
    __launch_bounds__(APPLY_THREADS) \
    __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : RLS_APPLY_WAVES)))

template <int PRO, int EPI, class R, class V>
__global__ void RLS_APPLY_BOUNDS_T(R) k_apply(ApplyArgsT<R, V> a) {
    extern __shared__ double lds_raw[];
    __shared__ double red[APPLY_THREADS];
    apply_body<PRO, EPI, R, V>(a, reinterpret_cast<R*>(lds_raw), red);
}

// dynamic LDS may use what the kernel's static LDS leaves of 160 KiB
static void allow_lds(const void* fn) {
    hipFuncAttributes attr;
    size_t stat = 0;
    if (hipFuncGetAttributes(&attr, fn) == hipSuccess) stat = attr.sharedSizeBytes;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(160 * 1024 - stat));
}

template <int PRO, int EPI, class R, class V>
static void launch_one(const ApplyArgsT<R, V>& a, hipStream_t s) {
    const TileShape T(a.g, EPI == EPI_RESTRICT);
    dim3 grid((a.g.nv + TILE_Y - 1) / TILE_Y, (a.g.nh + TILE_X - 1) / TILE_X,
              a.nslot);
    hipLaunchKernelGGL((k_apply<PRO, EPI, R, V>), grid, dim3(APPLY_THREADS),
                       sizeof(R) * T.lds_elems(), s, a);
}

// Every (prologue, epilogue) pair in use: all of them in FP64, the V-cycle's
// (and the plain product) in FP32, with FP32 or BF16 vectors.
#define RLS_APPLY_VARIANTS_F64(X)     \
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
#define RLS_APPLY_VARIANTS_F32(X)     \
    X(PRO_JACOBI, EPI_CHEB)           \
    X(PRO_JACOBI, EPI_RESTRICT)       \
    X(PRO_PROLONG, EPI_CHEB)          \
    X(PRO_PROLONG_JAC, EPI_CHEB)      \
    X(PRO_PLAIN, EPI_STORE)           \
    X(PRO_PLAIN, EPI_RESTRICT)        \
    X(PRO_PLAIN, EPI_CHEB)

void configure_apply_kernels() {
    static bool done = false;
    if (done) return;
#define RLS_CFG64(P, E) allow_lds((const void*)k_apply<P, E, double, double>);
#define RLS_CFG32(P, E) allow_lds((const void*)k_apply<P, E, float, float>);
#define RLS_CFG16(P, E) allow_lds((const void*)k_apply<P, E, float, bf16>);
    RLS_APPLY_VARIANTS_F64(RLS_CFG64)
    RLS_APPLY_VARIANTS_F32(RLS_CFG32)
    RLS_APPLY_VARIANTS_F32(RLS_CFG16)
#undef RLS_CFG64
#undef RLS_CFG32
#undef RLS_CFG16
    (void)hipGetLastError();
    done = true;
}

// Partial sums per slot of a level's kernels: one per tile, or one per
// workgroup of the sparse-level kernels.
int apply_tiles(const LevelGeom& g) {
    if (g.ct.on) return ct_parts((int64_t)g.nv * g.nh);
    return ((g.nv + TILE_Y - 1) / TILE_Y) * ((g.nh + TILE_X - 1) / TILE_X);
}

size_t apply_lds_bytes(const LevelGeom& g, int epi) {
    const TileShape T(g, epi == EPI_RESTRICT);
    return sizeof(double) * T.lds_elems();
}

size_t apply_lds_bytes(const LevelGeomT<float>& g, int epi) {
    const TileShape T(g, epi == EPI_RESTRICT);
    return sizeof(float) * T.lds_elems();
}

// Finest-level Chebyshev step: the tiled kernel with a compile-time band
// radius where it applies, the general kernel otherwise.
void launch_smooth_fine(const ApplyArgsT<double>& a, hipStream_t s) {
    if (!launch_smooth_fine_tiled(a, s))
        launch_one<PRO_PLAIN, EPI_CHEB, double>(a, s);
}
void launch_smooth_fine(const ApplyArgsT<float>& a, hipStream_t s) {
    if (!launch_smooth_fine_tiled(a, s))
        launch_one<PRO_PLAIN, EPI_CHEB, float>(a, s);
}
void launch_smooth_fine(const ApplyArgsT<float, bf16>& a, hipStream_t s) {
    if (!launch_smooth_fine_tiled(a, s))
        launch_one<PRO_PLAIN, EPI_CHEB, float, bf16>(a, s);
}

void launch_apply(int pro, int epi, const ApplyArgsT<double>& a, hipStream_t s) {
#define RLS_LAUNCH(P, E) \
    if (pro == P && epi == E) { launch_one<P, E, double>(a, s); return; }
    RLS_APPLY_VARIANTS_F64(RLS_LAUNCH)
#undef RLS_LAUNCH
    std::fprintf(stderr, "rls: no FP64 level-operator kernel for prologue %d, "
                         "epilogue %d\n", pro, epi);
    std::abort();
}

void launch_apply(int pro, int epi, const ApplyArgsT<float>& a, hipStream_t s) {
#define RLS_LAUNCH(P, E) \
    if (pro == P && epi == E) { launch_one<P, E, float>(a, s); return; }
    RLS_APPLY_VARIANTS_F32(RLS_LAUNCH)
#undef RLS_LAUNCH
    std::fprintf(stderr, "rls: no FP32 level-operator kernel for prologue %d, "
                         "epilogue %d\n", pro, epi);
    std::abort();
}

void launch_apply(int pro, int epi, const ApplyArgsT<float, bf16>& a,
                  hipStream_t s) {
#define RLS_LAUNCH(P, E) \
    if (pro == P && epi == E) { launch_one<P, E, float, bf16>(a, s); return; }
    RLS_APPLY_VARIANTS_F32(RLS_LAUNCH)
#undef RLS_LAUNCH
    std::fprintf(stderr, "rls: no BF16-vector level-operator kernel for "
                         "prologue %d, epilogue %d\n", pro, epi);
    std::abort();
}

}  // namespace rls
