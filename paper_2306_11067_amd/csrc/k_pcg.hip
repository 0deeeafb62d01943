// Batched preconditioned conjugate gradients: vector updates with FP64
// partial sums and the per-lambda scalar recurrences.  Reductions are
// deterministic: every workgroup writes one partial per slot, and a single
// workgroup per slot adds the partials in a fixed order.
#include <cmath>

#include "common.h"
#include "pcg_ctl.h"

namespace rls {

constexpr int VB = 256;          // threads per vector block
constexpr int VPT = 8;           // elements per thread
constexpr int VCHUNK = VB * VPT;

int vec_blocks(int64_t n) { return (int)((n + VCHUNK - 1) / VCHUNK); }

__global__ void k_broadcast(const double* __restrict__ src, int64_t n,
                            double* __restrict__ dst) {
    const int slot = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dst[(size_t)slot * n + p] = src[p];
}

// r = f - kx (f shared or per slot)
__global__ void k_axpy_sub(const double* __restrict__ f, int f_shared,
                           const double* __restrict__ kx, int64_t n,
                           double* __restrict__ r) {
    const int slot = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const size_t o = (size_t)slot * n + p;
    r[o] = f[f_shared ? p : o] - kx[o];
}

__global__ void __launch_bounds__(VB)
k_dot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
      const int* __restrict__ slots, const int* __restrict__ active,
      double* __restrict__ part) {
    __shared__ double sh[VB];
    const int slot = slots ? slots[blockIdx.y] : (int)blockIdx.y;
    if (active && !active[slot]) return;
    const size_t base = (size_t)slot * n;
    double s = 0.0;
    const int64_t p0 = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t p = p0 + (int64_t)k * VB;
        if (p < n) s += a[base + p] * b[base + p];
    }
    s = block_sum<VB>(s, sh);
    if (threadIdx.x == 0) part[(size_t)slot * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(VB)
k_sumsq(const double* __restrict__ a, int64_t n, double* __restrict__ part) {
    __shared__ double sh[VB];
    const int slot = blockIdx.y;
    const size_t base = (size_t)slot * n;
    double s = 0.0;
    const int64_t p0 = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t p = p0 + (int64_t)k * VB;
        if (p < n) s += a[base + p] * a[base + p];
    }
    s = block_sum<VB>(s, sh);
    if (threadIdx.x == 0) part[(size_t)slot * gridDim.x + blockIdx.x] = s;
}

// partial sums of (a_slot - b)^2, b shared by all slots
__global__ void __launch_bounds__(VB)
k_sub_sumsq(const double* __restrict__ a, const double* __restrict__ b,
            int64_t n, double* __restrict__ part) {
    __shared__ double sh[VB];
    const int slot = blockIdx.y;
    const size_t base = (size_t)slot * n;
    double s = 0.0;
    const int64_t p0 = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t p = p0 + (int64_t)k * VB;
        if (p < n) {
            const double t = a[base + p] - b[p];
            s += t * t;
        }
    }
    s = block_sum<VB>(s, sh);
    if (threadIdx.x == 0) part[(size_t)slot * gridDim.x + blockIdx.x] = s;
}

// partial sums of ||D L x||^2 over both gradient planes
__global__ void __launch_bounds__(VB)
k_weighted_grad_sq(const double* __restrict__ x, const double* __restrict__ d,
                   int nv, int nh, int periodic, double* __restrict__ part) {
    __shared__ double sh[VB];
    const int slot = blockIdx.y;
    const int64_t n = (int64_t)nv * nh;
    const double* xs = x + (size_t)slot * n;
    double s = 0.0;
    const int64_t p0 = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t p = p0 + (int64_t)k * VB;
        if (p >= n) continue;
        const int i = (int)(p % nv), j = (int)(p / nv);
        int ip = i + 1, jp = j + 1;
        if (wrap_or_drop(ip, nv, periodic)) {
            const double w = d ? d[p] : 1.0;
            const double t = w * (xs[ip + (int64_t)nv * j] - xs[p]);
            s += t * t;
        }
        if (wrap_or_drop(jp, nh, periodic)) {
            const double w = d ? d[n + p] : 1.0;
            const double t = w * (xs[i + (int64_t)nv * jp] - xs[p]);
            s += t * t;
        }
    }
    s = block_sum<VB>(s, sh);
    if (threadIdx.x == 0) part[(size_t)slot * gridDim.x + blockIdx.x] = s;
}

// alpha = gamma / (p . q) (folded finalization); x += alpha p ;
// r -= alpha q ; partial ||r||^2
__global__ void __launch_bounds__(VB)
k_update_xr(SlotState* __restrict__ st, int* __restrict__ active,
            const int* __restrict__ slots, int64_t n, double* __restrict__ x,
            double* __restrict__ r, const double* __restrict__ p,
            const double* __restrict__ q, const double* __restrict__ part_pq,
            int npq, int parity, double* __restrict__ part) {
    __shared__ double sh[VB];
    const int slot = slots ? slots[blockIdx.y] : (int)blockIdx.y;
    if (!active[slot]) return;
    double al;
    // block 0 of the slot's row of blocks leads
    if (!pcg_alpha<VB>(st, active, slot, part_pq, npq, parity, blockIdx.x == 0,
                       sh, al))
        return;
    const size_t base = (size_t)slot * n;
    double s = 0.0;
    const int64_t p0 = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t e = p0 + (int64_t)k * VB;
        if (e < n) {
            x[base + e] += al * p[base + e];
            const double rn = r[base + e] - al * q[base + e];
            r[base + e] = rn;
            s += rn * rn;
        }
    }
    s = block_sum<VB>(s, sh);
    if (threadIdx.x == 0) part[(size_t)slot * gridDim.x + blockIdx.x] = s;
}

__device__ double slot_sum(const double* part, int nparts, double* sh) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += VB) s += part[k];
    return block_sum<VB>(s, sh);
}

__global__ void __launch_bounds__(VB)
k_pcg_init(SlotState* __restrict__ st, const double* __restrict__ fparts,
           int nf, const double* __restrict__ rparts, int nr, double tol,
           int absolute, int maxit, int* __restrict__ active) {
    __shared__ double sh[VB];
    const int slot = blockIdx.x;
    const double ff = slot_sum(fparts, nf, sh);
    const double rr = slot_sum(rparts + (size_t)slot * nr, nr, sh);
    if (threadIdx.x == 0) {
        SlotState& s = st[slot];
        s.fnorm = sqrt(ff);
        s.target = absolute ? tol : tol * s.fnorm;
        s.rr = rr;
        s.gam[0] = s.gam[1] = 0.0;
        s.alpha = 0.0;
        s.it = 0;
        s.ncycle = 1;
        s.maxit = maxit;
        s.flags = 0;
        s.active = 1;
        if (!isfinite(rr)) {
            s.flags |= RLS_FLAG_NONFINITE;
            s.active = 0;
        } else if (sqrt(rr) <= s.target) {
            s.flags |= RLS_FLAG_CONVERGED;
            s.active = 0;
        }
        active[slot] = s.active;
    }
}

__global__ void __launch_bounds__(VB)
k_reduce_slots(const double* __restrict__ part, int nparts,
               double* __restrict__ out) {
    __shared__ double sh[VB];
    const int slot = blockIdx.x;
    const double s = slot_sum(part + (size_t)slot * nparts, nparts, sh);
    if (threadIdx.x == 0) out[slot] = s;
}

// ---- boundary of a reduced-precision V-cycle under flexible FP64 PCG -----

// Narrowing copy dst = (float) src over nslot slots (slot list optional).
__global__ void __launch_bounds__(VB)
k_to_f32(const double* __restrict__ src, int64_t n, const int* slots,
         float* __restrict__ dst) {
    const int slot = slots ? slots[blockIdx.y] : (int)blockIdx.y;
    const size_t base = (size_t)slot * n;
    const int64_t p0 = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t p = p0 + (int64_t)k * VB;
        if (p < n) dst[base + p] = (float)src[base + p];
    }
}

// Convergence test on ||r|| (as the FP64 path does in its first V-cycle
// kernel; skipped when st is null), then rlo = r rounded to the V-cycle's
// storage type V (float or bf16).
template <class V>
__global__ void __launch_bounds__(VB)
k_vc_enter(SlotState* st, int* active, const int* slots, const double* part_rr,
           int nrr, int64_t n, const double* __restrict__ r,
           V* __restrict__ rlo) {
    __shared__ double sh[VB];
    const int slot = slots ? slots[blockIdx.y] : (int)blockIdx.y;
    if (active && !active[slot]) return;
    if (st && !pcg_gate<VB>(st, active, slot, part_rr, nrr, blockIdx.x == 0, sh))
        return;
    const size_t base = (size_t)slot * n;
    const int64_t p0 = (int64_t)blockIdx.x * VCHUNK + threadIdx.x;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t p = p0 + (int64_t)k * VB;
        if (p < n) rlo[base + p] = Cvt<double, V>::out(r[base + p]);
    }
}

// z = zlo widened to FP64 and the partials of r . z and z . q ([slot][part],
// npart parts of n / npart consecutive points each).
template <class V>
__global__ void __launch_bounds__(VB)
k_vc_exit(const int* slots, const int* active, int64_t n, int npart,
          const V* __restrict__ zlo, double* __restrict__ z,
          const double* __restrict__ r, const double* __restrict__ q,
          double* part_rz, double* part_zq) {
    __shared__ double sh[VB];
    const int slot = slots ? slots[blockIdx.y] : (int)blockIdx.y;
    if (active && !active[slot]) return;
    const size_t base = (size_t)slot * n;
    const int64_t len = (n + npart - 1) / npart;
    const int64_t lo = (int64_t)blockIdx.x * len;
    const int64_t hi = lo + len < n ? lo + len : n;
    double rz = 0.0, zq = 0.0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += VB) {
        const double zv = Cvt<double, V>::in(zlo[base + p]);
        z[base + p] = zv;
        rz += r[base + p] * zv;
        if (q) zq += zv * q[base + p];
    }
    const double a = block_sum<VB>(rz, sh);
    if (threadIdx.x == 0) part_rz[(size_t)slot * npart + blockIdx.x] = a;
    if (part_zq) {
        const double b = block_sum<VB>(zq, sh);
        if (threadIdx.x == 0) part_zq[(size_t)slot * npart + blockIdx.x] = b;
    }
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_broadcast(const double* src, int64_t n, int nslot, double* dst,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_broadcast, dim3(nblk(n, 256), nslot), dim3(256), 0, s,
                       src, n, dst);
}
void launch_axpy_sub(const double* f, int f_shared, const double* kx,
                     int64_t n, int nslot, double* r, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_sub, dim3(nblk(n, 256), nslot), dim3(256), 0, s,
                       f, f_shared, kx, n, r);
}
void launch_dot(const double* a, const double* b, int64_t n, int nslot,
                const int* slots, const int* active, double* part,
                hipStream_t s) {
    hipLaunchKernelGGL(k_dot, dim3(vec_blocks(n), nslot), dim3(VB), 0, s, a, b,
                       n, slots, active, part);
}
void launch_sumsq_slots(const double* a, int64_t n, int nslot, double* part,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_sumsq, dim3(vec_blocks(n), nslot), dim3(VB), 0, s, a,
                       n, part);
}
void launch_sub_sumsq(const double* a, const double* b, int64_t n, int nslot,
                      double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_sumsq, dim3(vec_blocks(n), nslot), dim3(VB), 0, s,
                       a, b, n, part);
}
void launch_weighted_grad_sq(const double* x, const double* d, int nv, int nh,
                             int periodic, int nslot, double* part,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_weighted_grad_sq,
                       dim3(vec_blocks((int64_t)nv * nh), nslot), dim3(VB), 0,
                       s, x, d, nv, nh, periodic, part);
}
void launch_update_xr(SlotState* st, int* active, const int* slots,
                      int64_t n, int nslot, double* x, double* r,
                      const double* p, const double* q, const double* part_pq,
                      int npq, int parity, double* part_rr, hipStream_t s) {
    hipLaunchKernelGGL(k_update_xr, dim3(vec_blocks(n), nslot), dim3(VB), 0, s,
                       st, active, slots, n, x, r, p, q, part_pq, npq, parity,
                       part_rr);
}
void launch_pcg_init(SlotState* st, int nslot, const double* fparts, int nf,
                     const double* rparts, int nr, double tol, int absolute,
                     int maxit, int* active, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_init, dim3(nslot), dim3(VB), 0, s, st, fparts, nf,
                       rparts, nr, tol, absolute, maxit, active);
}
void launch_reduce_slots(const double* part, int nparts, int nslot,
                         double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_slots, dim3(nslot), dim3(VB), 0, s, part,
                       nparts, out);
}

void launch_to_f32(const double* src, int64_t n, int nslot, const int* slots,
                   float* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3(vec_blocks(n), nslot), dim3(VB), 0, s,
                       src, n, slots, dst);
}

template <class V>
void launch_vc_enter(SlotState* st, int* active, const int* slots, int nslot,
                     const double* part_rr, int nrr, int64_t n, const double* r,
                     V* rlo, hipStream_t s) {
    hipLaunchKernelGGL(k_vc_enter<V>, dim3(vec_blocks(n), nslot), dim3(VB), 0,
                       s, st, active, slots, part_rr, nrr, n, r, rlo);
}

template <class V>
void launch_vc_exit(const int* slots, const int* active, int nslot, int64_t n,
                    int npart, const V* zlo, double* z, const double* r,
                    const double* q, double* part_rz, double* part_zq,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_vc_exit<V>, dim3(npart, nslot), dim3(VB), 0, s, slots,
                       active, n, npart, zlo, z, r, q, part_rz, part_zq);
}

template void launch_vc_enter(SlotState*, int*, const int*, int, const double*,
                              int, int64_t, const double*, float*, hipStream_t);
template void launch_vc_enter(SlotState*, int*, const int*, int, const double*,
                              int, int64_t, const double*, bf16*, hipStream_t);
template void launch_vc_exit(const int*, const int*, int, int64_t, int,
                             const float*, double*, const double*,
                             const double*, double*, double*, hipStream_t);
template void launch_vc_exit(const int*, const int*, int, int64_t, int,
                             const bf16*, double*, const double*,
                             const double*, double*, double*, hipStream_t);

}  // namespace rls
