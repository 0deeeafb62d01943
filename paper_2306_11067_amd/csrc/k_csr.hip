// Sparse (CSR) forward operators: the tomography projector A and its
// one-sided multigrid hierarchy A_{k+1} = A_k P (paper Section 3.2), built
// and applied on the GPU.  Everything is deterministic: atomics are used
// only for integer counts, and every floating-point sum runs in a fixed
// order (sorted keys, fixed reduction trees).
#include <cstdint>

#include "common.h"

namespace rls {

constexpr int CSR_THREADS = 256;
constexpr int SORT_CAP = 4096;   // longest transposed row sorted in LDS
constexpr int COARSEN_CAP = 2048;  // longest expanded row (4 per nonzero)

// ---- exclusive prefix sum of int64 counts (one workgroup; setup only) ----
__global__ void __launch_bounds__(1024) k_scan_excl(const int64_t* cnt, int64_t n,
                                                   int64_t* out) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t lo = t * per, hi = lo + per < n ? lo + per : n;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        out[n] = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t i = lo; i < hi; ++i) {
        out[i] = acc;
        acc += cnt[i];
    }
}

// ---- transpose -----------------------------------------------------------
__global__ void k_col_count(const int* __restrict__ ci, int64_t nnz,
                            unsigned long long* cnt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[ci[e]], 1ull);
}

__global__ void k_scatter_t(const int64_t* __restrict__ rp,
                            const int* __restrict__ ci,
                            const double* __restrict__ va, int64_t m,
                            const int64_t* __restrict__ rpt,
                            unsigned long long* cursor, int* cit, double* vat) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        const int64_t pos = rpt[j] + (int64_t)atomicAdd(&cursor[j], 1ull);
        cit[pos] = (int)i;
        vat[pos] = va[e];
    }
}

// Bitonic sort of n (power of two) keys with values in LDS.
template <class K, class V>
__device__ void lds_bitonic(K* key, V* val, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (n >> 1); t += blockDim.x) {
                const int lo = 2 * stride * (t / stride) + (t % stride);
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                if ((key[lo] > key[hi]) == up) {
                    const K k = key[lo];
                    key[lo] = key[hi];
                    key[hi] = k;
                    const V v = val[lo];
                    val[lo] = val[hi];
                    val[hi] = v;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int pow2_at_least(int n) {
    int p = 2;
    while (p < n) p <<= 1;
    return p;
}

// Sort every row of a CSR by column (keys unique per row).
__global__ void __launch_bounds__(CSR_THREADS)
k_segment_sort(const int64_t* __restrict__ rp, int* ci, double* va, int* err) {
    __shared__ int key[SORT_CAP];
    __shared__ double val[SORT_CAP];
    const int64_t r = blockIdx.x;
    const int64_t b = rp[r], len = rp[r + 1] - b;
    if (len <= 1) return;
    if (len > SORT_CAP) {
        if (threadIdx.x == 0) atomicOr(err, 1);
        return;
    }
    const int n = pow2_at_least((int)len);
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        key[t] = t < len ? ci[b + t] : 0x7fffffff;
        val[t] = t < len ? va[b + t] : 0.0;
    }
    __syncthreads();
    lds_bitonic(key, val, n);
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
        ci[b + t] = key[t];
        va[b + t] = val[t];
    }
}

// ---- A_{k+1} = A_k P: expand, sort by coarse column, reduce --------------
// Coarse points of fine point f along one axis (vertex-centred linear
// interpolation; the last odd point copies, or wraps when periodic).
__device__ __forceinline__ int csr_interp(int f, int nf, int periodic, int* I,
                                          double* w) {
    const int nc = nf >> 1;
    if ((f & 1) == 0) { I[0] = f >> 1; w[0] = 1.0; return 1; }
    const int c = f >> 1;
    if (c + 1 < nc) { I[0] = c; I[1] = c + 1; w[0] = w[1] = 0.5; return 2; }
    if (periodic) { I[0] = c; I[1] = 0; w[0] = w[1] = 0.5; return 2; }
    I[0] = c; w[0] = 1.0; return 1;
}

// mode 0: cnt[row] = nonzeros of the coarse row; mode 1: write them at
// rpc[row] (columns ascending; equal columns summed in expansion order).
__global__ void __launch_bounds__(CSR_THREADS)
k_coarsen(const int64_t* __restrict__ rp, const int* __restrict__ ci,
          const double* __restrict__ va, int nvf, int nhf, int periodic,
          int mode, int64_t* cnt, const int64_t* rpc, int* cic, double* vac,
          int* err) {
    __shared__ unsigned long long key[COARSEN_CAP];
    __shared__ double val[COARSEN_CAP];
    __shared__ int head[COARSEN_CAP];
    const int64_t r = blockIdx.x;
    const int64_t b = rp[r], len = rp[r + 1] - b;
    const int nvc = nvf >> 1;
    if (len * 4 > COARSEN_CAP) {
        if (threadIdx.x == 0) atomicOr(err, 2);
        return;
    }
    // expansion: entry e of the row gives up to 4 slots 4e..4e+3
    const int ne = (int)len * 4;
    const int n = pow2_at_least(ne > 1 ? ne : 2);
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        key[t] = ~0ull;
        val[t] = 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < len; e += blockDim.x) {
        const int j = ci[b + e];
        const int fi = j % nvf, fj = j / nvf;
        int Ii[2], Jj[2];
        double wi[2], wj[2];
        const int ni = csr_interp(fi, nvf, periodic, Ii, wi);
        const int nj = csr_interp(fj, nhf, periodic, Jj, wj);
        const double a = va[b + e];
        int q = 0;
        for (int y = 0; y < nj; ++y)
            for (int x = 0; x < ni; ++x, ++q) {
                const unsigned long long J =
                    (unsigned long long)(Ii[x] + nvc * Jj[y]);
                key[4 * e + q] = (J << 16) | (unsigned long long)(4 * e + q);
                val[4 * e + q] = a * wi[x] * wj[y];
            }
    }
    __syncthreads();
    lds_bitonic(key, val, n);
    // segment heads over the valid prefix
    int nvalid = 0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const bool ok = key[t] != ~0ull;
        head[t] = ok && (t == 0 || (key[t] >> 16) != (key[t - 1] >> 16)) ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // inclusive running count of heads (serial: rows are short)
        int acc = 0;
        for (int t = 0; t < n; ++t) {
            if (key[t] == ~0ull) break;
            acc += head[t];
            head[t] = head[t] ? acc : -acc;   // >0: head with its rank
        }
        nvalid = acc;
        if (mode == 0) cnt[r] = acc;
    }
    if (mode == 0) return;
    __syncthreads();
    const int64_t out0 = rpc[r];
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        if (key[t] == ~0ull || head[t] <= 0) continue;
        double s = val[t];
        for (int u = t + 1; u < n && key[u] != ~0ull && head[u] < 0; ++u) s += val[u];
        const int rank = head[t] - 1;
        cic[out0 + rank] = (int)(key[t] >> 16);
        vac[out0 + rank] = s;
    }
    (void)nvalid;
}

// ---- per-column statistics from the transposed CSR ------------------------
// diag(A^T A)_j = sum_i A_ij^2
__global__ void k_row_sumsq(const int64_t* __restrict__ rpt,
                            const double* __restrict__ vat, int64_t n,
                            double* out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int64_t e = rpt[j]; e < rpt[j + 1]; ++e) s += vat[e] * vat[e];
    out[j] = s;
}

// ---- SpMV over lambda slots: y_s = A x_s (x = 1 when null) ----------------
// One wave per row; lanes stride the row; fixed-order wave reduction.
template <class VT, class XT, class YT>
__global__ void __launch_bounds__(CSR_THREADS)
k_spmv1(const int64_t* __restrict__ rp, const int* __restrict__ ci,
        const VT* __restrict__ va, int64_t nrows, int64_t xstride,
        const XT* __restrict__ x, int64_t ystride, YT* __restrict__ y,
        const int* slots, const int* active, int x_shared) {
    const int z = blockIdx.y;
    const int slot = slots ? slots[z] : z;
    if (active && !active[slot]) return;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (CSR_THREADS / 64) + (threadIdx.x >> 6);
    if (row >= nrows) return;
    const XT* xs = x ? x + (x_shared ? 0 : (size_t)slot * xstride) : nullptr;
    double s = 0.0;
    for (int64_t e = rp[row] + lane; e < rp[row + 1]; e += 64)
        s += (double)va[e] * (xs ? (double)xs[ci[e]] : 1.0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[(size_t)slot * ystride + row] = (YT)s;
}

// One wave per row and up to SPMV_SB slots (grid y: groups of SPMV_SB
// entries of the slot list): the row's columns and values are loaded once,
// SPMV_CH per lane at a time, and used for every slot of the group, so A is
// read once per group instead of once per slot.  Each lane accumulates its
// entries e = lane + 64 k in increasing k, then the same fixed-order wave
// reduction as k_spmv1: the two kernels give bit-identical results, and the
// launcher picks by the number of slots (the one-slot kernel keeps more
// loads in flight per row; the grouped one reads A fewer times).
constexpr int SPMV_SB = 8;
constexpr int SPMV_CH = 8;
// Smallest slot count that takes the grouped kernel (measured on the 256^2
// projector: 3 slots 67.5 vs 73.0 ms per PCG iteration, 4 slots 84.1 vs 80.7,
// 16 slots 305 vs 228).
constexpr int SPMV_GROUP_MIN = 4;
template <class VT, class XT, class YT>
__global__ void __launch_bounds__(CSR_THREADS)
k_spmv(const int64_t* __restrict__ rp, const int* __restrict__ ci,
       const VT* __restrict__ va, int64_t nrows, int64_t xstride,
       const XT* __restrict__ x, int64_t ystride, YT* __restrict__ y,
       int nslot, const int* slots, const int* active, int x_shared) {
    int sl[SPMV_SB];
    bool on[SPMV_SB];
    bool any = false;
#pragma unroll
    for (int j = 0; j < SPMV_SB; ++j) {
        const int z = blockIdx.y * SPMV_SB + j;
        on[j] = z < nslot;
        sl[j] = on[j] ? (slots ? slots[z] : z) : 0;
        if (on[j] && active && !active[sl[j]]) on[j] = false;
        any = any || on[j];
    }
    if (!any) return;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (CSR_THREADS / 64) + (threadIdx.x >> 6);
    if (row >= nrows) return;
    double acc[SPMV_SB];
#pragma unroll
    for (int j = 0; j < SPMV_SB; ++j) acc[j] = 0.0;
    const int64_t beg = rp[row], end = rp[row + 1];
    for (int64_t e0 = beg; e0 < end; e0 += 64 * SPMV_CH) {
        int c[SPMV_CH];
        double v[SPMV_CH];
#pragma unroll
        for (int k = 0; k < SPMV_CH; ++k) {
            const int64_t e = e0 + lane + 64 * k;
            const bool ok = e < end;
            c[k] = ok ? ci[e] : 0;
            v[k] = ok ? (double)va[e] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < SPMV_SB; ++j) {
            if (!on[j]) continue;
            const XT* xs = x ? x + (x_shared ? 0 : (size_t)sl[j] * xstride) : nullptr;
#pragma unroll
            for (int k = 0; k < SPMV_CH; ++k)
                if (e0 + lane + 64 * k < end)
                    acc[j] += v[k] * (xs ? (double)xs[c[k]] : 1.0);
        }
    }
#pragma unroll
    for (int j = 0; j < SPMV_SB; ++j) {
        double s = acc[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (on[j] && lane == 0) y[(size_t)sl[j] * ystride + row] = (YT)s;
    }
}

// ---- dense Gram of the coarsest operator: G = A_c^T A_c -------------------
// G(J1, J2) = sum_i A(i, J1) A(i, J2) by merging the sorted rows J1, J2 of
// A_c^T; one thread per pair J1 <= J2.
__global__ void k_dense_gram(const int64_t* __restrict__ rpt,
                             const int* __restrict__ cit,
                             const double* __restrict__ vat, int nc, double* G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nc * nc) return;
    const int J1 = (int)(e % nc), J2 = (int)(e / nc);
    if (J1 > J2) return;
    int64_t a = rpt[J1], ae = rpt[J1 + 1], b = rpt[J2], be = rpt[J2 + 1];
    double s = 0.0;
    while (a < ae && b < be) {
        const int ia = cit[a], ib = cit[b];
        if (ia == ib) {
            s += vat[a] * vat[b];
            ++a;
            ++b;
        } else if (ia < ib) {
            ++a;
        } else {
            ++b;
        }
    }
    G[J1 + (int64_t)nc * J2] = s;
    G[J2 + (int64_t)nc * J1] = s;
}

__global__ void k_f64_from_f32(const float* __restrict__ a, int64_t n,
                               double* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

// ---- host launchers --------------------------------------------------------
static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_scan_excl(const int64_t* cnt, int64_t n, int64_t* out,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, cnt, n, out);
}

void launch_csr_transpose_count(const int* ci, int64_t nnz,
                                unsigned long long* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_col_count, dim3(nb(nnz, 256)), dim3(256), 0, s, ci,
                       nnz, cnt);
}

void launch_csr_transpose_fill(const int64_t* rp, const int* ci,
                               const double* va, int64_t m, int64_t n,
                               const int64_t* rpt, unsigned long long* cursor,
                               int* cit, double* vat, int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_t, dim3(nb(m, 256)), dim3(256), 0, s, rp, ci,
                       va, m, rpt, cursor, cit, vat);
    hipLaunchKernelGGL(k_segment_sort, dim3((unsigned)n), dim3(CSR_THREADS), 0,
                       s, rpt, cit, vat, err);
}

void launch_csr_coarsen(const int64_t* rp, const int* ci, const double* va,
                        int64_t m, int nvf, int nhf, int periodic, int mode,
                        int64_t* cnt, const int64_t* rpc, int* cic,
                        double* vac, int* err, hipStream_t s) {
    hipLaunchKernelGGL(k_coarsen, dim3((unsigned)m), dim3(CSR_THREADS), 0, s,
                       rp, ci, va, nvf, nhf, periodic, mode, cnt, rpc, cic,
                       vac, err);
}

void launch_row_sumsq(const int64_t* rpt, const double* vat, int64_t n,
                      double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_row_sumsq, dim3(nb(n, 256)), dim3(256), 0, s, rpt,
                       vat, n, out);
}

template <class VT, class XT, class YT>
void launch_spmv(const int64_t* rp, const int* ci, const VT* va, int64_t nrows,
                 int64_t xstride, const XT* x, int x_shared, int64_t ystride,
                 YT* y, int nslot, const int* slots, const int* active,
                 hipStream_t s) {
    if (nslot >= SPMV_GROUP_MIN) {
        hipLaunchKernelGGL((k_spmv<VT, XT, YT>),
                           dim3(nb(nrows, CSR_THREADS / 64),
                                (nslot + SPMV_SB - 1) / SPMV_SB),
                           dim3(CSR_THREADS), 0, s, rp, ci, va, nrows, xstride,
                           x, ystride, y, nslot, slots, active, x_shared);
    } else {
        hipLaunchKernelGGL((k_spmv1<VT, XT, YT>),
                           dim3(nb(nrows, CSR_THREADS / 64), nslot),
                           dim3(CSR_THREADS), 0, s, rp, ci, va, nrows, xstride,
                           x, ystride, y, slots, active, x_shared);
    }
}
template void launch_spmv<double, double, double>(
    const int64_t*, const int*, const double*, int64_t, int64_t,
    const double*, int, int64_t, double*, int, const int*, const int*,
    hipStream_t);
template void launch_spmv<float, float, float>(
    const int64_t*, const int*, const float*, int64_t, int64_t, const float*,
    int, int64_t, float*, int, const int*, const int*, hipStream_t);

void launch_dense_gram(const int64_t* rpt, const int* cit, const double* vat,
                       int nc, double* G, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_gram, dim3(nb((int64_t)nc * nc, 256)),
                       dim3(256), 0, s, rpt, cit, vat, nc, G);
}

void launch_f64_from_f32(const float* a, int64_t n, double* b, hipStream_t s) {
    hipLaunchKernelGGL(k_f64_from_f32, dim3(nb(n, 256)), dim3(256), 0, s, a, n,
                       b);
}

}  // namespace rls
