// Setup kernels: lambda-free hierarchy (once per problem and per weighting)
// and per-sweep coarse data (Gershgorin bounds, Chebyshev coefficients,
// coarsest factorization).
//
// Paper anchors: the Galerkin coarse operators P^T K P and the one-sided
// hierarchy A_{k+1} = A_k P_k, M_{k+1} = M_k P_k of Section 3.2; the
// level diagonals diag(A_k^T A_k), diag(M_k^T M_k) of Section 3.2; the exact
// coarsest solve of Algorithm 1.  For the separable blur A = A_h (x) A_v and
// P = P_h (x) P_v, A_k^T A_k = (P_h^T..A_h^T A_h..P_h) (x) (same for v), so
// each level stores two 1D Gram bands instead of a 2D operator.
#include <cmath>

#include "common.h"

namespace rls {

// ---------------------------------------------------------------- 1D bands
// Band of the 1D blur (B x)_i = sum_t tap_t x(ext(i - t)), t = -r..r.
__global__ void k_blur_band(const double* __restrict__ taps, int r, int n,
                            int bc, double* __restrict__ band) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int w = 2 * r + 1;
    double* row = band + (size_t)i * w;
    for (int k = 0; k < w; ++k) row[k] = 0.0;
    const int map = bc == RLS_BC_PERIODIC ? MAP_WRAP
                  : bc == RLS_BC_REFLECTIVE ? MAP_REFLECT : MAP_ZERO;
    for (int t = -r; t <= r; ++t) {
        bool ok;
        const int c = map_index(i - t, n, map, ok);
        if (!ok) continue;
        int k;
        if (map == MAP_WRAP) {
            k = -t;                         // |t| <= r < n/2: no aliasing
        } else {
            k = c - i;                      // reflection stays within r
        }
        row[k + r] += taps[t + r];
    }
}

// out = band^T: entry (c, i) of the transpose is entry (i, c) of the band.
__global__ void k_transpose_band(const double* __restrict__ band, int n,
                                 int bw, int periodic,
                                 double* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int w = 2 * bw + 1;
    for (int k = -bw; k <= bw; ++k) {
        int i = c - k;
        double v = 0.0;
        if (wrap_or_drop(i, n, periodic)) v = band[(size_t)i * w + k + bw];
        out[(size_t)c * w + (-k) + bw] = v;
    }
}

// G = A^T A from the band of A (half width ra): G(i, i+k) =
// sum_m A(m, i) A(m, i+k), m = i + dm, |dm| <= ra.
__global__ void k_gram_band(const double* __restrict__ a, int n, int ra,
                            int periodic, double* __restrict__ g, int bwg) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int wg = 2 * bwg + 1, wa = 2 * ra + 1;
    if (idx >= n * wg) return;
    const int i = idx / wg;
    const int k = idx % wg - bwg;
    double s = 0.0;
    for (int dm = -ra; dm <= ra; ++dm) {
        int m = i + dm;
        if (!wrap_or_drop(m, n, periodic)) continue;
        const int o1 = -dm, o2 = k - dm;   // offsets of columns i, i+k in row m
        if (o2 < -ra || o2 > ra) continue;
        s += a[(size_t)m * wa + o1 + ra] * a[(size_t)m * wa + o2 + ra];
    }
    g[idx] = s;
}

// Coarse band G_c = P^T G P with the vertex-centred interpolation.
__global__ void k_galerkin_band(const double* __restrict__ gf, int nf,
                                int bwf, int periodic,
                                double* __restrict__ gc, int bwc) {
    const int nc = nf >> 1;
    const int wc = 2 * bwc + 1, wf = 2 * bwf + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nc * wc) return;
    const int I = idx / wc;
    const int K = idx % wc - bwc;
    int J = I + K;
    double s = 0.0;
    if (wrap_or_drop(J, nc, periodic)) {
        for (int a = -1; a <= 1; ++a) {
            int f = 2 * I + a;
            if (!wrap_or_drop(f, nf, periodic)) continue;
            const double pf = interp_weight(f, I, nf, periodic);
            if (pf == 0.0) continue;
            for (int b = -1; b <= 1; ++b) {
                // fine neighbour of coarse J, reached from f by offset o
                const int o = (2 * K + b) - a;   // (2J+b) - (2I+a) before wrap
                int gpt = 2 * I + 2 * K + b;
                if (!wrap_or_drop(gpt, nf, periodic)) continue;
                const double pg = interp_weight(gpt, J, nf, periodic);
                if (pg == 0.0) continue;
                if (o < -bwf || o > bwf) continue;
                s += pf * gf[(size_t)f * wf + o + bwf] * pg;
            }
        }
    }
    gc[idx] = s;
}

__global__ void k_band_stats(const double* __restrict__ band, int n, int bw,
                             double* __restrict__ diag,
                             double* __restrict__ rowabs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int w = 2 * bw + 1;
    double s = 0.0;
    for (int k = 0; k < w; ++k) s += fabs(band[(size_t)i * w + k]);
    diag[i] = band[(size_t)i * w + bw];
    rowabs[i] = s;
}

// ---------------------------------------------------------------- stencils
// Fine-level L^T D^2 L as a 5-point stencil in the five-plane layout.
__global__ void k_fine_stencil(const double* __restrict__ d, int nv, int nh,
                               int periodic, double* __restrict__ pl) {
    const int64_t n = (int64_t)nv * nh;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int i = (int)(idx % nv), j = (int)(idx / nv);
    auto wv = [&](int ii, int jj) -> double {   // weight^2 of edge (ii,jj)-(ii+1,jj)
        if (!periodic && ii >= nv - 1) return 0.0;
        if (!wrap_or_drop(ii, nv, periodic)) return 0.0;
        const double w = d ? d[ii + (int64_t)nv * jj] : 1.0;
        return w * w;
    };
    auto wh = [&](int ii, int jj) -> double {   // edge (ii,jj)-(ii,jj+1)
        if (!periodic && jj >= nh - 1) return 0.0;
        if (!wrap_or_drop(jj, nh, periodic)) return 0.0;
        const double w = d ? d[n + ii + (int64_t)nv * jj] : 1.0;
        return w * w;
    };
    const double a = wv(i, j), bdn = wv(i - 1, j), c = wh(i, j), e = wh(i, j - 1);
    pl[idx] = a + bdn + c + e;
    pl[n + idx] = -a;
    pl[2 * n + idx] = -c;
    pl[3 * n + idx] = 0.0;
    pl[4 * n + idx] = 0.0;
}

// Entry S(f, f + (di, dj)) of a five-plane stencil, zero outside a
// non-periodic grid.
__device__ __forceinline__ double stencil_entry(const double* __restrict__ pl,
                                                int nv, int nh, int periodic,
                                                int fi, int fj, int di,
                                                int dj) {
    const int64_t n = (int64_t)nv * nh;
    int gi = fi + di, gj = fj + dj;
    if (!wrap_or_drop(gi, nv, periodic) || !wrap_or_drop(gj, nh, periodic))
        return 0.0;
    int pi, pj, plane;
    // canonical owner of the coupling and its plane
    if (di == 0 && dj == 0) { pi = fi; pj = fj; plane = 0; }
    else if (di == 1 && dj == 0) { pi = fi; pj = fj; plane = 1; }
    else if (di == -1 && dj == 0) { pi = fi - 1; pj = fj; plane = 1; }
    else if (di == 0 && dj == 1) { pi = fi; pj = fj; plane = 2; }
    else if (di == 0 && dj == -1) { pi = fi; pj = fj - 1; plane = 2; }
    else if (di == 1 && dj == 1) { pi = fi; pj = fj; plane = 3; }
    else if (di == -1 && dj == -1) { pi = fi - 1; pj = fj - 1; plane = 3; }
    else if (di == -1 && dj == 1) { pi = fi; pj = fj; plane = 4; }
    else { pi = fi + 1; pj = fj - 1; plane = 4; }   // (1, -1)
    if (!wrap_or_drop(pi, nv, periodic) || !wrap_or_drop(pj, nh, periodic))
        return 0.0;
    return pl[plane * n + pi + (int64_t)nv * pj];
}

// Coarse stencil P^T S P (P = P_h (x) P_v), five planes.
__global__ void k_galerkin_stencil(const double* __restrict__ fp, int nvf,
                                   int nhf, int periodic,
                                   double* __restrict__ cp) {
    const int nvc = nvf >> 1, nhc = nhf >> 1;
    const int64_t nc = (int64_t)nvc * nhc;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nc) return;
    const int I = (int)(idx % nvc), J = (int)(idx / nvc);
    const int ti[5] = {0, 1, 0, 1, -1};
    const int tj[5] = {0, 0, 1, 1, 1};
    double acc[5] = {0, 0, 0, 0, 0};
    int TI[5], TJ[5];
    bool tok[5];
    for (int t = 0; t < 5; ++t) {
        TI[t] = I + ti[t];
        TJ[t] = J + tj[t];
        tok[t] = wrap_or_drop(TI[t], nvc, periodic) &&
                 wrap_or_drop(TJ[t], nhc, periodic);
    }
    for (int a = -1; a <= 1; ++a) {
        int fi = 2 * I + a;
        if (!wrap_or_drop(fi, nvf, periodic)) continue;
        const double wi = interp_weight(fi, I, nvf, periodic);
        if (wi == 0.0) continue;
        for (int b = -1; b <= 1; ++b) {
            int fj = 2 * J + b;
            if (!wrap_or_drop(fj, nhf, periodic)) continue;
            const double wj = interp_weight(fj, J, nhf, periodic);
            if (wj == 0.0) continue;
            const double pf = wi * wj;
            for (int di = -1; di <= 1; ++di) {
                for (int dj = -1; dj <= 1; ++dj) {
                    const double s = stencil_entry(fp, nvf, nhf, periodic, fi,
                                                   fj, di, dj);
                    if (s == 0.0) continue;
                    int gi = fi + di, gj = fj + dj;
                    if (!wrap_or_drop(gi, nvf, periodic) ||
                        !wrap_or_drop(gj, nhf, periodic))
                        continue;
                    for (int t = 0; t < 5; ++t) {
                        if (!tok[t]) continue;
                        const double pg = interp_weight(gi, TI[t], nvf, periodic) *
                                          interp_weight(gj, TJ[t], nhf, periodic);
                        if (pg != 0.0) acc[t] += pf * s * pg;
                    }
                }
            }
        }
    }
    for (int t = 0; t < 5; ++t) cp[t * nc + idx] = acc[t];
}

__global__ void k_stencil_rowabs(const double* __restrict__ pl, int nv, int nh,
                                 int periodic, double* __restrict__ ra) {
    const int64_t n = (int64_t)nv * nh;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int i = (int)(idx % nv), j = (int)(idx / nv);
    double s = 0.0;
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj)
            s += fabs(stencil_entry(pl, nv, nh, periodic, i, j, di, dj));
    ra[idx] = s;
}

// ---------------------------------------------------------------- per sweep
// rho = max_p (rowabs_G(p) + lam^2 rowabs_S(p)) / (diag_G(p) + lam^2 S_pp).
__global__ void __launch_bounds__(256)
k_gershgorin(LevelGeom g, const double* __restrict__ lam2,
             double* __restrict__ rho) {
    __shared__ double sh[256];
    const int slot = blockIdx.x;
    const double l2 = lam2[slot];
    const int64_t n = (int64_t)g.nv * g.nh;
    double m = 0.0;
    for (int64_t p = threadIdx.x; p < n; p += 256) {
        const int i = (int)(p % g.nv), j = (int)(p / g.nv);
        const double num = g.gv.rowabs[i] * g.gh.rowabs[j] + l2 * g.S.rowabs[p];
        const double den = g.gv.diag[i] * g.gh.diag[j] + l2 * g.S.c[p];
        m = fmax(m, num / den);
    }
    m = block_max<256>(m, sh);
    if (threadIdx.x == 0) rho[slot] = m;
}

// Chebyshev step coefficients on [rho/ratio, rho]: step 0 (c1, c2) =
// (0, 1/theta); step s >= 1: rho_s = 1/(2 sigma - rho_{s-1}),
// (c1, c2) = (rho_s rho_{s-1}, 2 rho_s / delta).
__global__ void k_cheb_coeffs(const double* __restrict__ rho, int nslot,
                              double ratio, int nu, int stride,
                              double* __restrict__ cheb) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= nslot) return;
    const double b = rho[slot], a = b / ratio;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
    const double sigma = theta / delta;
    double* c = cheb + (size_t)slot * stride;
    c[0] = 0.0;
    c[1] = 1.0 / theta;
    double rold = 1.0 / sigma;
    for (int s = 1; s < nu; ++s) {
        const double r = 1.0 / (2.0 * sigma - rold);
        c[2 * s] = r * rold;
        c[2 * s + 1] = 2.0 * r / delta;
        rold = r;
    }
}

// Dense coarsest operator G_h (x) G_v + lam^2 S, column-major, per slot.
__global__ void k_coarse_assemble(LevelGeom g, const double* __restrict__ lam2,
                                  double* __restrict__ Kc) {
    const int n = g.nv * g.nh;
    const int slot = blockIdx.y;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;   // column = row (sym.)
    if (col >= n) return;
    const double l2 = lam2[slot];
    double* K = Kc + (size_t)slot * n * n + (size_t)col * n;
    for (int r = 0; r < n; ++r) K[r] = 0.0;
    const int i = col % g.nv, j = col / g.nv;
    const int pv = g.gv.map == MAP_WRAP, ph = g.gh.map == MAP_WRAP;
    const int wv = 2 * g.gv.bw + 1, wh = 2 * g.gh.bw + 1;
    // K is symmetric: column `col` equals row `col`.
    for (int kh = -g.gh.bw; kh <= g.gh.bw; ++kh) {
        int jj = j + kh;
        if (!wrap_or_drop(jj, g.nh, ph)) continue;
        const double ch = g.gh.table[(size_t)j * wh + kh + g.gh.bw];
        if (ch == 0.0) continue;
        for (int kv = -g.gv.bw; kv <= g.gv.bw; ++kv) {
            int ii = i + kv;
            if (!wrap_or_drop(ii, g.nv, pv)) continue;
            K[ii + g.nv * jj] += g.gv.table[(size_t)i * wv + kv + g.gv.bw] * ch;
        }
    }
    const int periodic = g.S.periodic;
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj) {
            const double* planes = g.S.c;   // five planes are contiguous
            const double s = stencil_entry(planes, g.nv, g.nh, periodic, i, j,
                                           di, dj);
            if (s == 0.0) continue;
            int ii = i + di, jj = j + dj;
            wrap_or_drop(ii, g.nv, periodic);
            wrap_or_drop(jj, g.nh, periodic);
            K[ii + g.nv * jj] += l2 * s;
        }
}

// Gershgorin bound for a sparse level: rho = max_p (|A^T A| 1 + lam^2
// |S| 1)_p / K_pp, with A >= 0 so |A^T A| 1 = A^T (A 1).
__global__ void __launch_bounds__(256)
k_gershgorin_ct(LevelGeom g, const double* __restrict__ lam2,
                double* __restrict__ rho) {
    __shared__ double sh[256];
    const int slot = blockIdx.x;
    const double l2 = lam2[slot];
    const int64_t n = (int64_t)g.nv * g.nh;
    double m = 0.0;
    for (int64_t p = threadIdx.x; p < n; p += 256) {
        const double num = g.ct.rowabs[p] + l2 * g.S.rowabs[p];
        const double den = g.ct.diag[p] + l2 * g.S.c[p];
        m = fmax(m, num / den);
    }
    m = block_max<256>(m, sh);
    if (threadIdx.x == 0) rho[slot] = m;
}

// Dense coarsest operator A_c^T A_c + lam^2 S for a sparse level (the Gram
// G is lambda-free and formed once), column-major, per slot.
__global__ void k_coarse_assemble_ct(LevelGeom g, const double* __restrict__ G,
                                     const double* __restrict__ lam2,
                                     double* __restrict__ Kc) {
    const int n = g.nv * g.nh;
    const int slot = blockIdx.y;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n) return;
    const double l2 = lam2[slot];
    double* K = Kc + (size_t)slot * n * n + (size_t)col * n;
    for (int r = 0; r < n; ++r) K[r] = G[(size_t)col * n + r];
    const int i = col % g.nv, j = col / g.nv;
    const int periodic = g.S.periodic;
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj) {
            const double s = stencil_entry(g.S.c, g.nv, g.nh, periodic, i, j,
                                           di, dj);
            if (s == 0.0) continue;
            int ii = i + di, jj = j + dj;
            wrap_or_drop(ii, g.nv, periodic);
            wrap_or_drop(jj, g.nh, periodic);
            K[ii + g.nv * jj] += l2 * s;
        }
}

// Cholesky K = L L^T (in place, lower, column-major) and W = L^{-1}
// (row-major into `work`, transposed copy after it).  One block per slot.
// info[slot] = 0, or the 1-based index of the first non-positive pivot.
__global__ void __launch_bounds__(1024)
k_cholesky_inverse(double* __restrict__ Kc, int n, double* __restrict__ work,
                   int* __restrict__ info) {
    const int slot = blockIdx.x;
    double* A = Kc + (size_t)slot * n * n;          // A(i, j) = A[j*n + i]
    double* W = work + (size_t)slot * 2 * n * n;    // W(i, c) = W[i*n + c]
    double* Wt = W + (size_t)n * n;                 // Wt[c*n + i] = W(i, c)
    __shared__ int bad;
    __shared__ double piv;
    const int t = threadIdx.x, nt = blockDim.x;
    if (t == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (t == 0) {
            const double a = A[(size_t)k * n + k];
            if (!(a > 0.0) || !isfinite(a)) { if (!bad) bad = k + 1; piv = 1.0; }
            else piv = sqrt(a);
            A[(size_t)k * n + k] = piv;
        }
        __syncthreads();
        const double p = piv;
        for (int i = k + 1 + t; i < n; i += nt) A[(size_t)k * n + i] /= p;
        __syncthreads();
        for (int i = k + 1 + t; i < n; i += nt) {
            const double lik = A[(size_t)k * n + i];
            for (int j = k + 1; j <= i; ++j)
                A[(size_t)j * n + i] -= lik * A[(size_t)k * n + j];
        }
        __syncthreads();
    }
    // W = L^{-1}: row i of W from rows < i (L W = I).
    for (int i = 0; i < n; ++i) {
        const double lii = A[(size_t)i * n + i];
        for (int c = t; c < n; c += nt) {
            double s = (c == i) ? 1.0 : 0.0;
            if (c < i) {
                for (int m = c; m < i; ++m)
                    s -= A[(size_t)m * n + i] * W[(size_t)m * n + c];
            } else if (c > i) {
                s = 0.0;
            }
            W[(size_t)i * n + c] = s / lii;
        }
        __syncthreads();
    }
    for (int e = t; e < n * n; e += nt) {
        const int i = e / n, c = e % n;
        Wt[(size_t)c * n + i] = W[e];
    }
    if (t == 0) info[slot] = bad;
}

// Blocked variant for n a multiple of 16 on the FP64 matrix cores: the
// trailing updates of the right-looking factorization and the block
// products of W = L^{-1} run as 16 x 16 x 4 MFMA tiles (one wave per tile;
// operand A element (i, k) on lane 16 k + i, operand B element (k, j) on
// lane 16 k + j, result element (i, j) on lane 16 (i mod 4) + j, register
// i / 4).  Diagonal blocks are factored / inverted in LDS.  Same outputs
// as k_cholesky_inverse.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
k_cholesky_mfma(double* __restrict__ Kc, int n, double* __restrict__ work,
                int* __restrict__ info) {
    const int slot = blockIdx.x;
    double* A = Kc + (size_t)slot * n * n;          // A(i, j) = A[j*n + i]
    double* W = work + (size_t)slot * 2 * n * n;    // W(i, c) = W[i*n + c]
    double* Wt = W + (size_t)n * n;
    __shared__ double blk[16 * 17];
    __shared__ double winv[16 * 17];
    __shared__ int bad;
    __shared__ double piv;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int li = lane & 15, lk = lane >> 4;       // operand row/col, k group
    const int nb = n / 16;
    if (t == 0) bad = 0;
    __syncthreads();
    // ---- factorization ----------------------------------------------------
    for (int kb = 0; kb < nb; ++kb) {
        const int k0 = 16 * kb;
        {
            const int r = t & 15, c = t >> 4;
            blk[c * 17 + r] = A[(size_t)(k0 + c) * n + k0 + r];
        }
        __syncthreads();
        for (int c = 0; c < 16; ++c) {
            if (t == 0) {
                const double a = blk[c * 17 + c];
                if (!(a > 0.0) || !isfinite(a)) {
                    if (!bad) bad = k0 + c + 1;
                    piv = 1.0;
                } else {
                    piv = sqrt(a);
                }
                blk[c * 17 + c] = piv;
            }
            __syncthreads();
            if (t > c && t < 16) blk[c * 17 + t] /= piv;
            __syncthreads();
            {
                const int r = t & 15, cc = t >> 4;
                if (cc > c && r >= cc) blk[cc * 17 + r] -= blk[c * 17 + r] * blk[c * 17 + cc];
            }
            __syncthreads();
        }
        {
            const int r = t & 15, c = t >> 4;
            if (r >= c) A[(size_t)(k0 + c) * n + k0 + r] = blk[c * 17 + r];
        }
        // panel: L(i, k0:k0+16) = A(i, k0:k0+16) L_kk^{-T}
        for (int i = k0 + 16 + t; i < n; i += 256) {
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                double a = A[(size_t)(k0 + c) * n + i];
                for (int m = 0; m < c; ++m) a -= x[m] * blk[m * 17 + c];
                x[c] = a / blk[c * 17 + c];
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) A[(size_t)(k0 + c) * n + i] = x[c];
        }
        __syncthreads();
        // trailing update of the lower tiles (I, J), kb < J <= I < nb
        const int m = nb - kb - 1;
        const int ntile = m * (m + 1) / 2;
        for (int e = wave; e < ntile; e += 4) {
            int Ir = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while (Ir * (Ir + 1) / 2 > e) --Ir;
            while ((Ir + 1) * (Ir + 2) / 2 <= e) ++Ir;
            const int Jr = e - Ir * (Ir + 1) / 2;
            const int I = kb + 1 + Ir, J = kb + 1 + Jr;
            v4d acc;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[r] = A[(size_t)(16 * J + li) * n + 16 * I + lk + 4 * r];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const size_t col = (size_t)(k0 + 4 * kk + lk) * n;
                const double a = -A[col + 16 * I + li];
                const double b = A[col + 16 * J + li];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                A[(size_t)(16 * J + li) * n + 16 * I + lk + 4 * r] = acc[r];
        }
        __syncthreads();
    }
    // ---- W = L^{-1}, block row by block row --------------------------------
    for (int I = 0; I < nb; ++I) {
        const int i0 = 16 * I;
        {
            const int r = t & 15, c = t >> 4;
            blk[c * 17 + r] = r >= c ? A[(size_t)(i0 + c) * n + i0 + r] : 0.0;
        }
        __syncthreads();
        if (t < 16) {   // column t of L_II^{-1} by forward substitution
            const int c = t;
            for (int i = 0; i < 16; ++i) {
                double s = (i == c) ? 1.0 : 0.0;
                if (i > c)
                    for (int mm = c; mm < i; ++mm) s -= blk[mm * 17 + i] * winv[c * 17 + mm];
                winv[c * 17 + i] = i < c ? 0.0 : s / blk[i * 17 + i];
            }
        }
        __syncthreads();
        {   // W_II and the zero blocks right of it
            const int r = t & 15, c = t >> 4;
            W[(size_t)(i0 + r) * n + i0 + c] = winv[c * 17 + r];
            for (int cb = i0 + 16 + c; cb < n; cb += 16)
                W[(size_t)(i0 + r) * n + cb] = 0.0;
        }
        // W_IJ = -W_II sum_{K=J}^{I-1} L_IK W_KJ
        for (int J = wave; J < I; J += 4) {
            v4d S = {0.0, 0.0, 0.0, 0.0};
            for (int K = J; K < I; ++K) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int kr = 16 * K + 4 * kk + lk;
                    const double a = A[(size_t)kr * n + i0 + li];
                    const double b = W[(size_t)kr * n + 16 * J + li];
                    S = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, S, 0, 0, 0);
                }
            }
            // S(k, j) for k = 4 kk + lk sits in register kk of this lane
            v4d out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const double a = -winv[(4 * kk + lk) * 17 + li];
                out = __builtin_amdgcn_mfma_f64_16x16x4f64(a, S[kk], out, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                W[(size_t)(i0 + lk + 4 * r) * n + 16 * J + li] = out[r];
        }
        __syncthreads();
    }
    for (int e = t; e < n * n; e += 256) {
        const int i = e / n, c = e % n;
        Wt[(size_t)c * n + i] = W[e];
    }
    if (t == 0) info[slot] = bad;
}

__global__ void k_check_weights(const double* __restrict__ d, int64_t n,
                                int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = d[i];
    if (!(v >= 0.0) || !isfinite(v)) atomicOr(bad, 1);
}

// ---------------------------------------------------------------- launchers
static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_blur_band(const double* taps, int r, int n, int bc, double* band,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_blur_band, dim3(nblk(n, 128)), dim3(128), 0, s, taps,
                       r, n, bc, band);
}
void launch_transpose_band(const double* band, int n, int bw, int periodic,
                           double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_band, dim3(nblk(n, 128)), dim3(128), 0, s,
                       band, n, bw, periodic, out);
}
void launch_gram_band(const double* a, int n, int ra, int periodic, double* g,
                      int bwg, hipStream_t s) {
    const int64_t tot = (int64_t)n * (2 * bwg + 1);
    hipLaunchKernelGGL(k_gram_band, dim3(nblk(tot, 128)), dim3(128), 0, s, a, n,
                       ra, periodic, g, bwg);
}
void launch_galerkin_band(const double* gf, int nf, int bwf, int periodic,
                          double* gc, int bwc, hipStream_t s) {
    const int64_t tot = (int64_t)(nf / 2) * (2 * bwc + 1);
    hipLaunchKernelGGL(k_galerkin_band, dim3(nblk(tot, 128)), dim3(128), 0, s,
                       gf, nf, bwf, periodic, gc, bwc);
}
void launch_band_stats(const double* band, int n, int bw, double* diag,
                       double* rowabs, hipStream_t s) {
    hipLaunchKernelGGL(k_band_stats, dim3(nblk(n, 128)), dim3(128), 0, s, band,
                       n, bw, diag, rowabs);
}
void launch_fine_stencil(const double* d, int nv, int nh, int periodic,
                         double* planes, hipStream_t s) {
    hipLaunchKernelGGL(k_fine_stencil, dim3(nblk((int64_t)nv * nh, 256)),
                       dim3(256), 0, s, d, nv, nh, periodic, planes);
}
void launch_galerkin_stencil(const double* fp, int nvf, int nhf, int periodic,
                             double* cp, hipStream_t s) {
    hipLaunchKernelGGL(k_galerkin_stencil,
                       dim3(nblk((int64_t)(nvf / 2) * (nhf / 2), 128)),
                       dim3(128), 0, s, fp, nvf, nhf, periodic, cp);
}
void launch_stencil_rowabs(const double* pl, int nv, int nh, int periodic,
                           double* ra, hipStream_t s) {
    hipLaunchKernelGGL(k_stencil_rowabs, dim3(nblk((int64_t)nv * nh, 256)),
                       dim3(256), 0, s, pl, nv, nh, periodic, ra);
}
void launch_gershgorin(const LevelGeom& g, const double* lam2, int nslot,
                       double* rho, hipStream_t s) {
    hipLaunchKernelGGL(k_gershgorin, dim3(nslot), dim3(256), 0, s, g, lam2,
                       rho);
}
void launch_cheb_coeffs(const double* rho, int nslot, double ratio, int nu,
                        int stride, double* cheb, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_coeffs, dim3(nblk(nslot, 64)), dim3(64), 0, s,
                       rho, nslot, ratio, nu, stride, cheb);
}
void launch_coarse_assemble(const LevelGeom& g, const double* lam2, int nslot,
                            double* Kc, hipStream_t s) {
    const int n = g.nv * g.nh;
    hipLaunchKernelGGL(k_coarse_assemble, dim3(nblk(n, 128), nslot), dim3(128),
                       0, s, g, lam2, Kc);
}
void launch_gershgorin_ct(const LevelGeom& g, const double* lam2, int nslot,
                          double* rho, hipStream_t s) {
    hipLaunchKernelGGL(k_gershgorin_ct, dim3(nslot), dim3(256), 0, s, g, lam2,
                       rho);
}
void launch_coarse_assemble_ct(const LevelGeom& g, const double* G,
                               const double* lam2, int nslot, double* Kc,
                               hipStream_t s) {
    const int n = g.nv * g.nh;
    hipLaunchKernelGGL(k_coarse_assemble_ct, dim3(nblk(n, 128), nslot),
                       dim3(128), 0, s, g, G, lam2, Kc);
}
void launch_cholesky_inverse(double* Kc, int n, int nslot, double* work,
                             int* info, hipStream_t s) {
    if (n % 16 == 0)
        hipLaunchKernelGGL(k_cholesky_mfma, dim3(nslot), dim3(256), 0, s, Kc, n,
                           work, info);
    else
        hipLaunchKernelGGL(k_cholesky_inverse, dim3(nslot), dim3(1024), 0, s,
                           Kc, n, work, info);
}
void launch_cholesky_inverse_scalar(double* Kc, int n, int nslot, double* work,
                                    int* info, hipStream_t s) {
    hipLaunchKernelGGL(k_cholesky_inverse, dim3(nslot), dim3(1024), 0, s, Kc,
                       n, work, info);
}
void launch_check_weights(const double* d, int64_t n, int* bad,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_check_weights, dim3(nblk(n, 256)), dim3(256), 0, s, d,
                       n, bad);
}

}  // namespace rls
