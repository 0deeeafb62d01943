// Device helpers shared by the kernels: index maps, interpolation weights,
// deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "rls_internal.h"

namespace rls {

// Position j of a 1D axis of length n under an index map; `ok` is false for
// a zero-extended position outside [0, n).
__device__ __forceinline__ int map_index(int j, int n, int map, bool& ok) {
    ok = true;
    if (j >= 0 && j < n) return j;
    if (map == MAP_WRAP) {
        j %= n;
        return j < 0 ? j + n : j;
    }
    if (map == MAP_REFLECT) {      // half-sample symmetric, period 2n
        int m = j % (2 * n);
        if (m < 0) m += 2 * n;
        return m < n ? m : 2 * n - 1 - m;
    }
    ok = false;
    return 0;
}

// Wrap (periodic) or reject (non-periodic) an index.
__device__ __forceinline__ bool wrap_or_drop(int& j, int n, int periodic) {
    if (j >= 0 && j < n) return true;
    if (!periodic) return false;
    j %= n;
    if (j < 0) j += n;
    return true;
}

// Weight of coarse point I in the vertex-centred linear interpolation to
// fine point f (fine size nf = 2 nc).  Coarse I sits on fine 2I; odd fine
// 2c+1 averages c and c+1; the last odd point wraps to coarse 0 when
// periodic and copies coarse nc-1 otherwise.  f and I are already in range.
__device__ __forceinline__ double interp_weight(int f, int I, int nf,
                                                int periodic) {
    const int nc = nf >> 1;
    if ((f & 1) == 0) return (f >> 1) == I ? 1.0 : 0.0;
    const int c = f >> 1;
    if (c + 1 < nc) return (I == c || I == c + 1) ? 0.5 : 0.0;
    if (periodic) return (I == c || I == 0) ? 0.5 : 0.0;
    return I == c ? 1.0 : 0.0;
}

// Sum of `v` over a block of BLOCK threads, fixed order.  Result valid in
// thread 0.  `sh` needs BLOCK doubles.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

}  // namespace rls
