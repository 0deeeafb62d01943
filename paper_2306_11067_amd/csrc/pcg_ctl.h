// Per-lambda PCG scalar recurrences, evaluated redundantly by every
// workgroup of the kernel that needs them.  Each workgroup adds the same
// partial sums in the same order, so all workgroups take the same decision
// without a separate finalization kernel; only the leader (first workgroup)
// writes the slot state, and never a field that another workgroup of the
// same kernel reads.  The caller says which workgroup of the slot leads
// (the grid dimension that indexes slots differs between kernels).
#pragma once

#include <cmath>

#include "common.h"

namespace rls {

// Sum of part[0..nparts) by a whole block, fixed order; every thread gets
// the result.  `sh` needs BLOCK doubles.
template <int BLOCK>
__device__ __forceinline__ double block_sum_parts(const double* part,
                                                  int nparts, double* sh) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += BLOCK) s += part[k];
    sh[threadIdx.x] = s;
    __syncthreads();
#pragma unroll
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ void stop_slot(SlotState* st, int* active, int slot,
                                          int flag) {
    st[slot].flags |= flag;
    st[slot].active = 0;
    active[slot] = 0;
}

// gamma_k = r_k . z_k from the V-cycle partials; beta_k = gamma_k /
// gamma_{k-1} (0 at the first iteration).  With part_zq (flexible CG, for a
// preconditioner that is not exactly the same linear map at every
// iteration) the Polak-Ribiere form z_k . (r_k - r_{k-1}) / gamma_{k-1} is
// used; since r_k - r_{k-1} = -alpha_{k-1} q_{k-1} it equals
// -alpha_{k-1} (z_k . q_{k-1}) / gamma_{k-1}.  Returns false when the slot
// stops (r . z not positive or not finite).
template <int BLOCK>
__device__ __forceinline__ bool pcg_beta(SlotState* st, int* active, int slot,
                                         const double* part_rz, int nrz,
                                         int parity, const double* part_zq,
                                         bool leader_block, double* sh,
                                         double& beta) {
    const double g = block_sum_parts<BLOCK>(part_rz + (size_t)slot * nrz, nrz, sh);
    const bool lead = leader_block && threadIdx.x == 0;
    if (!isfinite(g) || !(g > 0.0)) {
        if (lead) stop_slot(st, active, slot,
                            isfinite(g) ? RLS_FLAG_BREAKDOWN : RLS_FLAG_NONFINITE);
        return false;
    }
    if (st[slot].it == 0) {
        beta = 0.0;
    } else if (part_zq) {
        const double zq =
            block_sum_parts<BLOCK>(part_zq + (size_t)slot * nrz, nrz, sh);
        beta = -st[slot].alpha * zq / st[slot].gam[parity];
    } else {
        beta = g / st[slot].gam[parity];
    }
    if (lead) st[slot].gam[1 - parity] = g;
    return true;
}

// alpha_k = gamma_k / (p_k . q_k); the leader counts the iteration.
template <int BLOCK>
__device__ __forceinline__ bool pcg_alpha(SlotState* st, int* active, int slot,
                                          const double* part_pq, int npq,
                                          int parity, bool leader_block,
                                          double* sh, double& alpha) {
    const double pq = block_sum_parts<BLOCK>(part_pq + (size_t)slot * npq, npq, sh);
    const bool lead = leader_block && threadIdx.x == 0;
    if (!isfinite(pq) || !(pq > 0.0)) {
        if (lead) stop_slot(st, active, slot,
                            isfinite(pq) ? RLS_FLAG_BREAKDOWN : RLS_FLAG_NONFINITE);
        return false;
    }
    alpha = st[slot].gam[1 - parity] / pq;
    if (lead) {
        st[slot].alpha = alpha;
        st[slot].it += 1;
    }
    return true;
}

// Convergence test on ||r_{k+1}|| before the V-cycle.  Returns false when
// the slot stops (converged, iteration cap, non-finite).
template <int BLOCK>
__device__ __forceinline__ bool pcg_gate(SlotState* st, int* active, int slot,
                                         const double* part_rr, int nrr,
                                         bool leader_block, double* sh) {
    const double rr = block_sum_parts<BLOCK>(part_rr + (size_t)slot * nrr, nrr, sh);
    const bool lead = leader_block && threadIdx.x == 0;
    int flag = 0;
    if (!isfinite(rr)) flag = RLS_FLAG_NONFINITE;
    else if (sqrt(rr) <= st[slot].target) flag = RLS_FLAG_CONVERGED;
    else if (st[slot].it >= st[slot].maxit) flag = RLS_FLAG_MAXIT;
    if (lead) st[slot].rr = rr;
    if (flag) {
        if (lead) stop_slot(st, active, slot, flag);
        return false;
    }
    if (lead) st[slot].ncycle += 1;
    return true;
}

}  // namespace rls
