// Finest-level Chebyshev smoothing step, specialised for a compile-time band
// radius.  This is the step the V-cycle (paper Algorithm 1, smoothing on the
// finest level) repeats most often: with the plain prologue and the
// Chebyshev epilogue it computes, per lambda slot,
//     d <- c1 d + c2 (f - K x) / diag(K),   x_out = x + d,
// with K = G_h (x) G_v + lambda^2 S (paper Section 3.2: the separable Gram
// of the blur plus the five-point stencil of L^T D^2 L on the fine grid).
// In FP64 and FP32 a run of these steps takes the equivalent three-term form
//     x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 (f - K x_k) / diag(K),
// which reads x_k, x_{k-1} and f and writes x_{k+1} over x_{k-1} (32 bytes
// per pixel instead of 40: d is never stored).
//
// It applies when both Gram bands of the level are uniform (one row of taps
// plus a wrap or reflection index map), the stencil has five points and the
// grid is a whole number of 64 x 16 tiles; the level-operator kernel covers
// every other case with the same arithmetic.
//
// Differences from the general kernel, all aimed at fewer instructions per
// output point:
//   * the band radius BW is a template parameter: the tap loops unroll, and
//     the taps (symmetric, so BW + 1 per direction) sit in scalar registers;
//   * the tile and its halo are loaded as units of 16 bytes of one row
//     (VEC consecutive columns, one load per column, one 16-byte LDS write),
//     spread evenly over the 256 threads, with branch-free wrap / reflect
//     index maps;
//   * the vertical pass gives every thread 4 consecutive rows of one column,
//     so all four waves work, and its results stay in registers: the
//     stencil term and the Chebyshev update follow directly, with 16-byte
//     global loads and stores of the 4 rows.
#include <type_traits>

#include "common.h"

namespace rls {
namespace {

constexpr int FY = 64;    // output rows per tile (contiguous axis)
constexpr int FX = 16;    // output columns per tile
constexpr int FZ = FINE_ZMAX;   // most slots per launch (inline slot list)
// Without a measured choice (ApplyArgsT::fine_nt), launches with at most
// this many slots use 512-thread workgroups: with one workgroup per CU the
// passes then run on two waves per SIMD.  Measured at
// 512 x 512, one PCG iteration with graph replay: one slot 2.54 ms against
// 2.62 (FP64) and 2.36 against 2.39 (FP32 V-cycle); two slots 3.34 against
// 3.39 (FP64) but 2.88 against 2.68 (FP32).
constexpr int FWIDE_MAX = 1;
constexpr int FBW = 20;   // largest band radius with a specialised kernel

template <class R>
struct Vec16;
template <>
struct Vec16<double> {
    using T = double2;
};
template <>
struct Vec16<float> {
    using T = float4;
};

// Tile geometry for band radius BW and NT threads (256: 8 horizontal
// outputs and 4 vertical outputs per thread; 512: 4 and 2).
template <class R, int BW, int NT>
struct FineShape {
    static constexpr int HWO = NT == 256 ? 8 : 4;      // horizontal outputs
    static constexpr int VWO = NT == 256 ? 4 : 2;      // vertical outputs
    static constexpr int VEC = 16 / (int)sizeof(R);   // elements per 16 bytes
    static constexpr int RY = FY + 2 * BW;            // input rows
    static constexpr int CX = FX + 2 * BW;            // input columns
    // Row stride of the input tile and column stride of the horizontal-pass
    // result: whole 16-byte units, an odd number of them, so that eight
    // lanes reading 16 bytes each at that stride hit eight distinct groups
    // of four LDS banks.
    static constexpr int SX = (((CX + VEC - 1) / VEC) | 1) * VEC;
    static constexpr int SH = (((RY + VEC - 1) / VEC) | 1) * VEC;
    static constexpr int NU = RY * (CX / VEC);        // load units
    static constexpr int UPT = (NU + NT - 1) / NT;    // units per thread
    static constexpr int HWL = HWO + 2 * BW;          // horizontal window
    static constexpr int VWL = VWO + 2 * BW;          // vertical window
    // vertical windows start at multiples of VWO rows: 16-byte reads when
    // that is a multiple of VEC, else 8-byte reads
    static constexpr int VCW = VWO % VEC == 0 ? VEC : 8 / (int)sizeof(R);
    static constexpr int NH = (FX / HWO) * RY;        // horizontal items
    // input tile, horizontal-pass result, diag G_v of the tile's rows
    static constexpr size_t lds_bytes =
        sizeof(R) * ((size_t)RY * SX + (size_t)FX * SH + FY);
    static_assert(BW % 2 == 0, "even band radius");
    static_assert(CX % VEC == 0, "whole load units per row");
    static_assert(HWL % VEC == 0 && VWL % VCW == 0, "whole vector windows");
    static_assert(NH <= NT, "one horizontal item per thread");
    static_assert((FY / VWO) * FX == NT, "one vertical item per thread");
};

// Everything one launch reads from its kernel arguments, packed into a few
// scalar-cache lines so that they arrive in one batch (the general argument
// block spreads them over a kilobyte, and the compiler fetches it line by
// line between branches).
template <class R, class V>
struct FineArgs {
    const V* in;            // x of every slot (storage type V)
    V* out;                 // x + d
    V* d;                   // Chebyshev direction, in place
    const V* f;             // right-hand side
    const R* sn;            // stencil planes: north, east couplings
    const R* se;
    const R* dv;            // diag G_v (nv), diag G_h (nh)
    const R* dh;
    const double* lam2;     // per slot
    const double* cheb;     // per slot (c1, c2) of this step
    const int* active;      // per slot, may be null
    double* part;           // partial sums of f . out [slot][tile]
    int nv, nh;
    int wrapv, wraph, per, f_shared;
    int cheb_stride, dot, part_stride;
    // 0: read d, store d; 1: read d, store no d; 2: d = x_in - x_prev with
    // x_prev read from out (overwritten in place by x_out), store no d
    int xmode;
    int zslot[FZ];          // slot of grid z
    // half tap rows plus centre (the Gram rows are symmetric), padded to the
    // kernel's radius: entry k is the coefficient at offset k - BW
    R tv[FBW + 1];
    R th[FBW + 1];
};

// Position x in [-n, 2n) of an axis of length n under the band's index map:
// periodic wrap, or half-sample reflection.
__device__ __forceinline__ int fine_map(int x, int n, bool wrap) {
    const int lo = wrap ? x + n : -1 - x;
    const int hi = wrap ? x - n : 2 * n - 1 - x;
    return x < 0 ? lo : (x >= n ? hi : x);
}

// Four consecutive elements at an element index aligned to four elements
// (16 bytes for FP32 and FP64, 8 for BF16), converted to R.
template <class R>
__device__ __forceinline__ void ld4(const R* base, uint32_t idx, R (&o)[4]) {
    const char* p =
        reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(R);
    if constexpr (sizeof(R) == 8) {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 16);
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    } else {
        const float4 a = *reinterpret_cast<const float4*>(p);
        o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    }
}
template <class R>
__device__ __forceinline__ void ld4(const bf16* base, uint32_t idx,
                                    R (&o)[4]) {
    const uint2 a = *reinterpret_cast<const uint2*>(
        reinterpret_cast<const char*>(base) + idx * 2u);
    o[0] = (R)__uint_as_float(a.x << 16);
    o[1] = (R)__uint_as_float(a.x & 0xffff0000u);
    o[2] = (R)__uint_as_float(a.y << 16);
    o[3] = (R)__uint_as_float(a.y & 0xffff0000u);
}

template <class R>
__device__ __forceinline__ void st4(R* base, uint32_t idx, const R (&v)[4]) {
    char* p = reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(R);
    if constexpr (sizeof(R) == 8) {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2*>(p + 16) = make_double2(v[2], v[3]);
    } else {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
}
template <class R>
__device__ __forceinline__ void st4(bf16* base, uint32_t idx,
                                    const R (&v)[4]) {
    uint32_t h[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) h[o] = float_to_bf16((float)v[o]).bits;
    *reinterpret_cast<uint2*>(reinterpret_cast<char*>(base) + idx * 2u) =
        make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

// Two consecutive elements at an even element index, converted to R.
template <class R>
__device__ __forceinline__ void ld2(const R* base, uint32_t idx, R (&o)[2]) {
    const char* p =
        reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(R);
    if constexpr (sizeof(R) == 8) {
        const double2 a = *reinterpret_cast<const double2*>(p);
        o[0] = a.x; o[1] = a.y;
    } else {
        const float2 a = *reinterpret_cast<const float2*>(p);
        o[0] = a.x; o[1] = a.y;
    }
}
template <class R>
__device__ __forceinline__ void ld2(const bf16* base, uint32_t idx,
                                    R (&o)[2]) {
    const uint32_t a = *reinterpret_cast<const uint32_t*>(
        reinterpret_cast<const char*>(base) + idx * 2u);
    o[0] = (R)__uint_as_float(a << 16);
    o[1] = (R)__uint_as_float(a & 0xffff0000u);
}
template <class R>
__device__ __forceinline__ void st2(R* base, uint32_t idx, const R (&v)[2]) {
    char* p = reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(R);
    if constexpr (sizeof(R) == 8)
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    else
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
}
template <class R>
__device__ __forceinline__ void st2(bf16* base, uint32_t idx,
                                    const R (&v)[2]) {
    *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) + idx * 2u) =
        (uint32_t)float_to_bf16((float)v[0]).bits |
        ((uint32_t)float_to_bf16((float)v[1]).bits << 16);
}
// N = 2 or 4 consecutive elements
template <class R, class T, int N>
__device__ __forceinline__ void ldn(const T* base, uint32_t idx, R (&o)[N]) {
    if constexpr (N == 4) ld4(base, idx, o);
    else ld2(base, idx, o);
}
template <class R, class T, int N>
__device__ __forceinline__ void stn(T* base, uint32_t idx, const R (&v)[N]) {
    if constexpr (N == 4) st4(base, idx, v);
    else st2(base, idx, v);
}

template <class R, class V>
__device__ __forceinline__ R ldg(const V* base, uint32_t idx) {
    return Cvt<R, V>::in(*reinterpret_cast<const V*>(
        reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(V)));
}

// N consecutive LDS elements read CW at a time (CW * sizeof(R) = 16 or 8
// bytes, the address aligned to that).
template <class R, int N, int CW = 16 / (int)sizeof(R)>
__device__ __forceinline__ void lds_window(const R* p, R (&w)[N]) {
    static_assert(N % CW == 0, "whole chunks");
    if constexpr (CW * sizeof(R) == 16) {
        using V = typename Vec16<R>::T;
#pragma unroll
        for (int m = 0; m < N / CW; ++m) {
            const V x = reinterpret_cast<const V*>(p)[m];
            if constexpr (CW == 2) {
                w[2 * m] = x.x; w[2 * m + 1] = x.y;
            } else {
                w[4 * m] = x.x; w[4 * m + 1] = x.y;
                w[4 * m + 2] = x.z; w[4 * m + 3] = x.w;
            }
        }
    } else {   // 8-byte chunks of two floats
        static_assert(CW == 2 && sizeof(R) == 4, "8-byte chunks of FP32");
#pragma unroll
        for (int m = 0; m < N / 2; ++m) {
            const float2 x = reinterpret_cast<const float2*>(p)[m];
            w[2 * m] = x.x; w[2 * m + 1] = x.y;
        }
    }
}

// The value of lane l - 1 of the same row of 16 lanes (DPP row shift; lane
// 0 of a row receives zero).
__device__ __forceinline__ int row_shr1_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
}
__device__ __forceinline__ double row_shr1(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = row_shr1_i((int)(b & 0xffffffffLL));
    const int hi = row_shr1_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) |
                                (long long)(unsigned)lo);
}
__device__ __forceinline__ float row_shr1(float v) {
    return __int_as_float(row_shr1_i(__float_as_int(v)));
}
// The value of lane l - 16 of the wave (lanes 0..15 receive their own).
__device__ __forceinline__ double shfl_up16(double v) {
    return __shfl_up(v, 16, 64);
}
__device__ __forceinline__ float shfl_up16(float v) {
    return __shfl_up(v, 16, 64);
}

template <class R, class V, int BW, int NT>
__global__ void __launch_bounds__(NT)
k_smooth_fine(FineArgs<R, V> a) {
    using S = FineShape<R, BW, NT>;
    constexpr int HWO = S::HWO, VWO = S::VWO;
    using VT = typename Vec16<R>::T;   // 16 bytes of R
    extern __shared__ __align__(16) double lds_raw[];
    __shared__ double red[NT];
    R* vin = reinterpret_cast<R*>(lds_raw);      // RY x SX, row-major
    R* ht = vin + S::RY * S::SX;                 // FX x SH, column-major
    R* dgl = ht + FX * S::SH;                    // FY: diag G_v, rows i0..
    const int t = threadIdx.x;
    const int z = blockIdx.z;
    // no branch may precede the argument loads (the compiler would fetch
    // the rest of the block after it): the slot list is always inline, and
    // the XCD-aware tile order of the general kernel is selected by a mask
    const int slot = a.zslot[z & (FZ - 1)];
    const int nv = a.nv, nh = a.nh;
    // An empty statement that takes arguments the vector loads need: the
    // scalar loads of the argument block issue before it, then one wait.
    // To the compiler it stands for a memory write, so the per-slot values
    // read below become vector loads: those complete in order, and waiting
    // for them does not wait for other scalar loads.
    R tv[BW + 1], th[BW + 1];
#pragma unroll
    for (int k = 0; k <= BW; ++k) {
        tv[k] = a.tv[k];
        th[k] = a.th[k];
    }
    asm volatile("" ::"s"(a.in), "s"(a.sn), "s"(slot), "s"(nv));
    const R l2 = (R)a.lam2[slot];
    const R cd = (R)a.cheb[(size_t)slot * a.cheb_stride];
    const R cr = (R)a.cheb[(size_t)slot * a.cheb_stride + 1];
    const int ntx = nv / FY, nty = nh / FX, ntile = ntx * nty;   // the grid
    const int tlin = blockIdx.x + ntx * blockIdx.y;
    const int keep = -(int)((ntile & 7) != 0);
    const int tile = (tlin & keep) |
                     (((tlin & 7) * (ntile >> 3) + (tlin >> 3)) & ~keep);
    const int tx = tile % ntx, ty = tile / ntx;
    const int i0 = tx * FY, j0 = ty * FX;
    const size_t so = (size_t)slot * ((size_t)nv * nh);
    const V* src = a.in + so;
    const V* f = a.f_shared ? a.f : a.f + so;
    V* dir = a.d + so;
    V* out = a.out + so;
    const bool wrapv = a.wrapv, wraph = a.wraph;
    const int per = a.per;

    // 1. operands of this thread's four outputs (rows r0..r0+3 of column c),
    //    requested first: right-hand side, direction, diagonals, couplings.
    const int c = t & (FX - 1), r0 = VWO * (t >> 4);
    const int gi0 = i0 + r0, gj = j0 + c;
    const uint32_t p0 = (uint32_t)gi0 + (uint32_t)nv * (uint32_t)gj;
    // The centre coupling is not read: on the finest level the stencil is
    // L^T D^2 L, whose rows sum to zero, so it is minus the sum of the four
    // couplings.  The west couplings (east couplings one column left) come
    // from the neighbouring lane, the south coupling of the first row (north
    // coupling one row down) from the lane 16 below; only the lanes at the
    // tile's left column and at a wave's first row group load them (wrapped
    // on a periodic grid, zero across a non-periodic edge).  diag G_v of the
    // tile's 64 rows is loaded once per tile into LDS.
    const int lane = t & 63;
    R pf[VWO], pd[VWO], psn[VWO], pse[VWO], psw[VWO], dgr[4];
    ldn(f, p0, pf);
    // direction of the last step, or (three-term form) the previous iterate
    ldn(a.xmode == 2 ? (const V*)out : (const V*)dir, p0, pd);
    ldn(a.sn, p0, psn);
    ldn(a.se, p0, pse);
    const R dgh = a.dh[gj];
    R pss0 = R(0);
#pragma unroll
    for (int o = 0; o < VWO; ++o) psw[o] = R(0);
#pragma unroll
    for (int o = 0; o < 4; ++o) dgr[o] = R(0);
    if (lane < 16) {
        if (gi0 > 0) pss0 = ldg<R>(a.sn, p0 - 1);
        else if (per) pss0 = ldg<R>(a.sn, (uint32_t)(nv - 1) + (uint32_t)nv * gj);
    }
    if (c == 0) {
        if (gj > 0) ldn(a.se, p0 - (uint32_t)nv, psw);
        else if (per)
            ldn(a.se, (uint32_t)gi0 + (uint32_t)nv * (uint32_t)(nh - 1), psw);
    }
    if (t < FY / 4) ld4(a.dv, (uint32_t)(i0 + 4 * t), dgr);

    // 2. the tile plus its halo of BW rows and columns, as units of VEC
    //    consecutive columns of one row, all loads in flight at once.  Unit
    //    e = t + NT k sits at row ii = e mod RY, column VEC (e div RY);
    //    interior tiles need no index map.
    R u[S::UPT][S::VEC];
    const bool inner = i0 >= BW && i0 + FY + BW <= nv && j0 >= BW &&
                       j0 + FX + BW <= nh;
    int ii = t % S::RY, jq = t / S::RY;
    constexpr int DI = NT % S::RY, DJ = NT / S::RY;
    if (inner) {
        const V* sb = src + (size_t)(i0 - BW) + (size_t)nv * (size_t)(j0 - BW);
#pragma unroll
        for (int k = 0; k < S::UPT; ++k) {
            const uint32_t o = (uint32_t)ii + (uint32_t)nv * (uint32_t)(jq * S::VEC);
#pragma unroll
            for (int cc = 0; cc < S::VEC; ++cc)
                u[k][cc] = t + NT * k < S::NU
                               ? ldg<R>(sb, o + (uint32_t)nv * (uint32_t)cc)
                               : R(0);
            ii += DI;
            jq += DJ;
            if (ii >= S::RY) { ii -= S::RY; ++jq; }
        }
    } else {
#pragma unroll
        for (int k = 0; k < S::UPT; ++k) {
            const uint32_t gi = (uint32_t)fine_map(i0 - BW + ii, nv, wrapv);
#pragma unroll
            for (int cc = 0; cc < S::VEC; ++cc) {
                u[k][cc] = R(0);
                if (t + NT * k < S::NU) {
                    const int gjj =
                        fine_map(j0 - BW + jq * S::VEC + cc, nh, wraph);
                    u[k][cc] = ldg<R>(src, gi + (uint32_t)nv * (uint32_t)gjj);
                }
            }
            ii += DI;
            jq += DJ;
            if (ii >= S::RY) { ii -= S::RY; ++jq; }
        }
    }
    // A slot that stopped inside a replayed chunk is skipped (its loads
    // above are harmless, its stores are not).  The flag's load queues
    // behind the tile loads, so waiting for it costs no more than the wait
    // for the tile that follows anyway.
    if (a.active && !a.active[slot]) return;
    if (t < FY / 4) {
#pragma unroll
        for (int o = 0; o < 4; ++o) dgl[4 * t + o] = dgr[o];
    }
#pragma unroll
    for (int k = 0; k < S::UPT; ++k) {
        const int e = t + NT * k;
        if (e < S::NU) {
            const int ii = e % S::RY, jq = e / S::RY;
            VT x;
            if constexpr (S::VEC == 2) {
                x.x = u[k][0]; x.y = u[k][1];
            } else {
                x.x = u[k][0]; x.y = u[k][1]; x.z = u[k][2]; x.w = u[k][3];
            }
            *reinterpret_cast<VT*>(vin + ii * S::SX + jq * S::VEC) = x;
        }
    }
    __syncthreads();

    // 3. horizontal pass over the tile's columns and every input row:
    //    ht(q, cc) = sum_k G_h(k) v(q, cc + k), k = 0..2BW
    if (t < S::NH) {
#pragma clang fp contract(off)
        const int hsel = t / S::RY;
        const int q = t - hsel * S::RY;
        const int c0 = hsel * HWO;
        R w[S::HWL];
        lds_window<R, S::HWL>(vin + q * S::SX + c0, w);
        R acc[HWO];
#pragma unroll
        for (int o = 0; o < HWO; ++o) acc[o] = th[BW] * w[o + BW];
#pragma unroll
        for (int k = 0; k < BW; ++k)
#pragma unroll
            for (int o = 0; o < HWO; ++o)
                acc[o] = fma(th[k], w[o + k] + w[o + 2 * BW - k], acc[o]);
#pragma unroll
        for (int o = 0; o < HWO; ++o) ht[(c0 + o) * S::SH + q] = acc[o];
    }
    __syncthreads();

    // 4. vertical pass for rows r0..r0+3 of column c
    R kv[VWO];
    {
#pragma clang fp contract(off)
        R w[S::VWL];
        lds_window<R, S::VWL, S::VCW>(ht + c * S::SH + r0, w);
#pragma unroll
        for (int o = 0; o < VWO; ++o) kv[o] = tv[BW] * w[o + BW];
#pragma unroll
        for (int k = 0; k < BW; ++k)
#pragma unroll
            for (int o = 0; o < VWO; ++o)
                kv[o] = fma(tv[k], w[o + k] + w[o + 2 * BW - k], kv[o]);
    }

    // 5. stencil term, Chebyshev update, stores
    const R* vc = vin + (r0 + BW) * S::SX + c + BW;
    R colv[VWO + 2];
#pragma unroll
    for (int o = 0; o < VWO + 2; ++o) colv[o] = vc[(o - 1) * S::SX];
    {
        const R up = shfl_up16(psn[VWO - 1]);
        if (lane >= 16) pss0 = up;
#pragma unroll
        for (int o = 0; o < VWO; ++o) {
            const R left = row_shr1(pse[o]);
            if (c != 0) psw[o] = left;
        }
    }
    R nd[VWO], nx[VWO];
    double prod[VWO];
#pragma unroll
    for (int o = 0; o < VWO; ++o) {
        // Every fused multiply-add is written out and nothing else is fused,
        // so both thread counts round every output the same way.
#pragma clang fp contract(off)
        const R v = colv[o + 1];
        const R ss = o == 0 ? pss0 : psn[o - 1];
        const R sc = -(((psn[o] + ss) + pse[o]) + psw[o]);
        R sv = fma(psn[o], colv[o + 2], sc * v);
        sv = fma(ss, colv[o], sv);
        sv = fma(pse[o], vc[o * S::SX + 1], sv);
        sv = fma(psw[o], vc[o * S::SX - 1], sv);
        const R kvo = fma(l2, sv, kv[o]);
        const R dg = fma(dgl[r0 + o], dgh, l2 * sc);
        const R dk = a.xmode == 2 ? v - pd[o] : pd[o];
        nd[o] = fma(cd, dk, cr * (pf[o] - kvo) / dg);
        nx[o] = v + nd[o];
        // rounded product (never fused into the sum below: the lane that
        // adds it may not be the lane that formed it)
        prod[o] = __dmul_rn((double)pf[o], (double)nx[o]);
    }
    if (a.xmode == 0) stn(dir, p0, nd);
    stn(out, p0, nx);
    if (a.dot) {
        // Partial of f . x_out over the tile in one order for both thread
        // counts (so a slot's result does not depend on how many slots the
        // launch has): the 1024 products go to LDS (over the input tile,
        // which is no longer read), 256 threads each sum 4 consecutive rows
        // of one column in row order, then a fixed tree.
        static_assert(S::lds_bytes >= sizeof(double) * FY * FX,
                      "room for the products");
        __syncthreads();
        double* pl = reinterpret_cast<double*>(lds_raw);
#pragma unroll
        for (int o = 0; o < VWO; ++o) pl[c * FY + r0 + o] = prod[o];
        __syncthreads();
        if (t < 256) {
            const int cc = t & (FX - 1), rr = 4 * (t >> 4);
            double dot = 0.0;
#pragma unroll
            for (int o = 0; o < 4; ++o)
                dot = __dadd_rn(dot, pl[cc * FY + rr + o]);
            red[t] = dot;
        }
        __syncthreads();
#pragma unroll
        for (int st = 128; st > 0; st >>= 1) {
            if (t < st) red[t] += red[t + st];
            __syncthreads();
        }
        if (t == 0) a.part[(size_t)slot * a.part_stride + tile] = red[0];
    }
}

bool aligned16(const void* p) {
    return ((uintptr_t)p & 15) == 0;
}

template <class R, class V>
int fine_radius(const ApplyArgsT<R, V>& a) {
    const LevelGeomT<R>& g = a.g;
    if (g.ct.on || !g.gv.uniform || !g.gh.uniform || g.S.nine) return -1;
    if (g.gv.map == MAP_ZERO || g.gh.map == MAP_ZERO) return -1;
    if (g.nv % FY != 0 || g.nh % FX != 0) return -1;
    if (!a.in || !a.out || !a.d || !a.f || !a.cheb || !a.lam2) return -1;
    if (!g.gv.htaps || !g.gh.htaps) return -1;
    // the slot of grid z comes from the inline list or is z itself
    if (a.nslot > FZ || (a.slots && a.zn != a.nslot)) return -1;
    const void* ptrs[] = {a.in, a.out, a.d, a.f, g.S.cn, g.S.ce, g.gv.diag};
    for (const void* p : ptrs)
        if (!aligned16(p)) return -1;
    int bw = g.gv.bw > g.gh.bw ? g.gv.bw : g.gh.bw;
    bw += bw & 1;
    if (bw < 2) bw = 2;
    return bw <= FBW ? bw : -1;
}

template <class R, class V>
FineArgs<R, V> fine_args(const ApplyArgsT<R, V>& a, int bw) {
    const LevelGeomT<R>& g = a.g;
    FineArgs<R, V> f{};
    f.in = a.in;
    f.out = a.out;
    f.d = a.d;
    f.f = a.f;
    f.sn = g.S.cn;
    f.se = g.S.ce;
    f.dv = g.gv.diag;
    f.dh = g.gh.diag;
    for (int k = 0; k <= FBW; ++k) {
        const int kv = k - (bw - g.gv.bw), kh = k - (bw - g.gh.bw);
        f.tv[k] = k <= bw && kv >= 0 ? g.gv.htaps[kv] : R(0);
        f.th[k] = k <= bw && kh >= 0 ? g.gh.htaps[kh] : R(0);
    }
    f.lam2 = a.lam2;
    f.cheb = a.cheb;
    f.active = a.active;
    f.part = a.part;
    f.nv = g.nv;
    f.nh = g.nh;
    f.wrapv = g.gv.map == MAP_WRAP;
    f.wraph = g.gh.map == MAP_WRAP;
    f.per = g.S.periodic;
    f.f_shared = a.f_shared;
    f.cheb_stride = a.cheb_stride;
    f.dot = a.dot;
    f.part_stride = a.part_stride;
    // the three-term form where x is stored in the arithmetic type (FP64,
    // FP32): forming the direction from two stored iterates then adds
    // rounding of the size each stored iterate already carries.  BF16
    // vectors keep the stored direction.
    constexpr bool xform = std::is_same<R, V>::value;
    f.xmode = xform && a.fine_xstep >= 0 ? (a.fine_xstep == 0 ? 1 : 2) : 0;
    for (int i = 0; i < FZ; ++i)
        f.zslot[i] = i < a.zn ? a.zslot[i] : i < a.nslot ? i : 0;
    return f;
}

// Dynamic LDS beyond the default 64 KiB needs the kernel attribute (the
// widest FP64 instances: 61 KiB of tile plus 4 KiB of static LDS).
template <class R, class V, int BW, int NT>
void allow_fine_lds() {
    static const bool done = [] {
        const void* fn = (const void*)k_smooth_fine<R, V, BW, NT>;
        hipFuncAttributes attr;
        size_t stat = 0;
        if (hipFuncGetAttributes(&attr, fn) == hipSuccess)
            stat = attr.sharedSizeBytes;
        (void)hipFuncSetAttribute(fn,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(160 * 1024 - stat));
        (void)hipGetLastError();
        return true;
    }();
    (void)done;
}

template <class R, class V, int BW>
void launch_fine(const ApplyArgsT<R, V>& a, hipStream_t s) {
    allow_fine_lds<R, V, BW, 256>();
    allow_fine_lds<R, V, BW, 512>();
    dim3 grid(a.g.nv / FY, a.g.nh / FX, a.nslot);
    const int nt = a.fine_nt ? a.fine_nt : a.nslot <= FWIDE_MAX ? 512 : 256;
    if (nt == 512)
        hipLaunchKernelGGL((k_smooth_fine<R, V, BW, 512>), grid, dim3(512),
                           (FineShape<R, BW, 512>::lds_bytes), s,
                           fine_args(a, BW));
    else
        hipLaunchKernelGGL((k_smooth_fine<R, V, BW, 256>), grid, dim3(256),
                           (FineShape<R, BW, 256>::lds_bytes), s,
                           fine_args(a, BW));
}

template <class R, class V>
bool fine_impl(const ApplyArgsT<R, V>& a, hipStream_t s) {
    switch (fine_radius(a)) {
        case 2: launch_fine<R, V, 2>(a, s); return true;
        case 4: launch_fine<R, V, 4>(a, s); return true;
        case 6: launch_fine<R, V, 6>(a, s); return true;
        case 8: launch_fine<R, V, 8>(a, s); return true;
        case 10: launch_fine<R, V, 10>(a, s); return true;
        case 12: launch_fine<R, V, 12>(a, s); return true;
        case 14: launch_fine<R, V, 14>(a, s); return true;
        case 16: launch_fine<R, V, 16>(a, s); return true;
        case 18: launch_fine<R, V, 18>(a, s); return true;
        case 20: launch_fine<R, V, 20>(a, s); return true;
        default: return false;
    }
}

}  // namespace

bool launch_smooth_fine_tiled(const ApplyArgsT<double>& a, hipStream_t s) {
    return fine_impl(a, s);
}
bool launch_smooth_fine_tiled(const ApplyArgsT<float>& a, hipStream_t s) {
    return fine_impl(a, s);
}
bool launch_smooth_fine_tiled(const ApplyArgsT<float, bf16>& a, hipStream_t s) {
    return fine_impl(a, s);
}

}  // namespace rls
