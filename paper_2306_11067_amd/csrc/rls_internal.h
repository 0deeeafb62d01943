// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rls.h"

namespace rls {

// Index extension of a 1D direction when reading outside [0, n).
enum MapKind : int { MAP_ZERO = 0, MAP_WRAP = 1, MAP_REFLECT = 2 };

// BF16 storage element: the upper half of an IEEE FP32 value.  Stores round
// to nearest, ties to even; finite values beyond the BF16 range become
// infinities, as IEEE rounding prescribes.
struct bf16 {
    uint16_t bits;
};
__host__ __device__ inline float bf16_to_float(bf16 x) {
    return __builtin_bit_cast(float, (uint32_t)x.bits << 16);
}
__host__ __device__ inline bf16 float_to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16{(uint16_t)(u >> 16)};
}

// Conversions between a storage type V and an arithmetic type R.
template <class R, class V>
struct Cvt {
    __host__ __device__ static R in(V v) { return (R)v; }
    __host__ __device__ static V out(R r) { return (V)r; }
};
template <class R>
struct Cvt<R, bf16> {
    __host__ __device__ static R in(bf16 v) { return (R)bf16_to_float(v); }
    __host__ __device__ static bf16 out(R r) { return float_to_bf16((float)r); }
};

// Arithmetic type of the V-cycle for a vector storage type.
template <class V>
struct CompOf {
    using T = V;
};
template <>
struct CompOf<bf16> {
    using T = float;
};

// A banded n x n operator along one image axis.  Row r, offset k in
// [-bw, bw] is the coefficient of x(map(r + k)).  `uniform` rows all equal
// `taps` (the index map supplies the boundary); otherwise `table` holds
// every row, with zeros where r + k falls outside a non-wrapping axis.
// R is the value type (double; float copies serve the FP32 V-cycle).
template <class R>
struct BandDevT {
    int n = 0;
    int bw = 0;
    int map = MAP_ZERO;
    int uniform = 0;
    const R* taps = nullptr;    // 2bw+1
    const R* table = nullptr;   // n * (2bw+1)
    const R* diag = nullptr;    // n
    const R* rowabs = nullptr;  // n: sum_k |row r|
    // host copy of the uniform row (2bw+1 values; host code only), for
    // kernels that take the taps in their arguments
    const R* htaps = nullptr;
};

// Galerkin stencil of L^T D^2 L on one level, five planes of n values:
// c (centre), cn (i+1, j), ce (i, j+1), cne (i+1, j+1), cse (i-1, j+1).
template <class R>
struct StencilDevT {
    const R* c = nullptr;
    const R* cn = nullptr;
    const R* ce = nullptr;
    const R* cne = nullptr;
    const R* cse = nullptr;
    const R* rowabs = nullptr;  // sum_j |S_ij|
    int nine = 0;               // 0: cne/cse are identically zero
    int periodic = 0;
};

// A level whose A_k^T A_k is applied through a sparse A_k (tomography):
// A_k (m x n_k) and A_k^T as CSR, column statistics, and the workspace of
// one application (shared by all levels, sized for the finest).
template <class R>
struct CsrDevT {
    int on = 0;
    int64_t m = 0;
    const int64_t* rp = nullptr;    // A_k
    const int* ci = nullptr;
    const R* va = nullptr;
    const int64_t* rpt = nullptr;   // A_k^T
    const int* cit = nullptr;
    const R* vat = nullptr;
    const R* diag = nullptr;        // diag(A_k^T A_k)
    const double* rowabs = nullptr; // A_k^T A_k 1 (A_k >= 0 entrywise)
    R* v = nullptr;                 // [slot][n_k] operand after the prologue
    R* y = nullptr;                 // [slot][m]   A_k v
    R* t = nullptr;                 // [slot][n_k] A_k^T y
    R* res = nullptr;               // [slot][n_k] residual before restriction
};

template <class R>
struct LevelGeomT {
    int nv = 0, nh = 0;
    BandDevT<R> gv, gh;         // separable Gram G_h (x) G_v
    StencilDevT<R> S;
    CsrDevT<R> ct;              // sparse A_k instead of the bands (ct.on)
};

using BandDev = BandDevT<double>;
using StencilDev = StencilDevT<double>;
using LevelGeom = LevelGeomT<double>;

// Tile of the level-operator kernel (i is the contiguous axis).
constexpr int TILE_Y = 64;
constexpr int TILE_X = 16;
constexpr int APPLY_THREADS = 256;

// Prologue: how the operand v of K v is formed while loading a tile.
enum Prologue : int {
    PRO_PLAIN = 0,    // v = in
    PRO_PUPDATE = 1,  // v = z + beta * p_old ; p_new = v (interior)
    PRO_JACOBI = 2,   // v = c2 f / diag(K): first Chebyshev step from zero
    PRO_PROLONG = 3,  // v = in + P e_coarse: coarse-grid correction
    PRO_PROLONG_JAC = 4  // v = c2 f / diag(K) + P e_coarse (nu = 1)
};
// Epilogue: what is done with (v, K v) at each output point.
enum Epilogue : int {
    EPI_STORE = 0,    // out = K v
    EPI_DOT = 1,      // out = K v ; partial sum of v . K v
    EPI_RESID = 2,    // out = f - K v
    EPI_CHEB = 3,     // d = c1 d + c2 (f - K v) / diag ; out = v + d
                      //   (optional partial sum of f . out)
    EPI_RESTRICT = 4  // fc = P^T (f - K v) on the coarse grid
};

struct SlotState {
    double gam[2];  // r . z of the last two iterations (double-buffered so
                    // that one kernel can read the old value while its
                    // leader writes the new one)
    double alpha;
    double rr;      // ||r||^2
    double target;  // residual norm target
    double fnorm;   // ||A^T b||
    int it;         // completed iterations
    int ncycle;     // V-cycles run (the initial one included)
    int active;
    int flags;
    int maxit;
};

// Slot lists up to this length also travel in the kernel arguments (read
// through the scalar kernel-argument path instead of a global load).
constexpr int ZINLINE = 32;
// Most slots in one launch of the tiled finest-level Chebyshev kernel (its
// slot list is inline).
constexpr int FINE_ZMAX = 64;

// Arguments of the level-operator kernel; R is the arithmetic type and the
// type of the level's bands and stencil (double, or float for the FP32 and
// BF16 V-cycles), V the storage type of its vectors (R, or bf16).  Per-slot
// scalars, Chebyshev coefficients and partial sums are always double.
template <class R, class V = R>
struct ApplyArgsT {
    LevelGeomT<R> g;
    int nslot = 0;                   // grid z: number of slots launched
    const int* slots = nullptr;      // slot of each grid z (null: identity)
    int zn = 0;                      // zn == nslot: zslot holds the list
    int zslot[ZINLINE] = {};
    const double* lam2 = nullptr;    // per slot lambda^2
    const int* active = nullptr;     // per slot, may be null (all active)
    const V* in = nullptr;           // v, z (PUPDATE) or x (PROLONG)
    const V* pold = nullptr;         // PRO_PUPDATE
    V* pnew = nullptr;               // PRO_PUPDATE
    const double* beta = nullptr;    // PRO_PUPDATE, per slot
    const V* ec = nullptr;           // PRO_PROLONG coarse correction
    V* out = nullptr;
    const V* f = nullptr;            // right-hand side (RESID/CHEB/RESTRICT/JACOBI)
    int f_shared = 0;                // f has one vector for all slots
    V* d = nullptr;                  // EPI_CHEB direction, in place
    const double* cheb = nullptr;    // per slot (c1, c2) of this step
    const double* cheb_first = nullptr;  // PRO_JACOBI: (c1, c2) of step 0
    int cheb_stride = 0;             // doubles between slots in cheb
    V* fc = nullptr;                 // EPI_RESTRICT coarse right-hand side
    int dot = 0;                     // EPI_CHEB: accumulate f . out
    double* part = nullptr;          // partial sums [slot][tile]
    int part_stride = 0;             // tiles per slot in part
    // PCG control folded into the kernels (see k_pcg.hip):
    SlotState* st = nullptr;
    int* active_w = nullptr;         // writable copy of `active` (leaders)
    const double* part_rz = nullptr; // PRO_PUPDATE: partials of r . z
    int nrz = 0;
    int parity = 0;                  // iteration parity (gam double buffer)
    int flex = 0;                    // PRO_PUPDATE: flexible (Polak-Ribiere) beta
    const double* part_zq = nullptr; // flex: partials of z_new . q_old
    int gate = 0;                    // convergence test before the V-cycle
    const double* part_rr = nullptr; // gate: partials of ||r||^2
    int nrr = 0;
    // threads per workgroup of the tiled finest-level Chebyshev kernel
    // (256 or 512, both giving the same results; 0: built-in rule)
    int fine_nt = 0;
    // position of this step in a run of consecutive tiled steps (-1:
    // not in such a run).  Those steps use the three-term form of the
    // recurrence: the first reads the direction d the previous (general)
    // step stored, the others form it as x_k - x_{k-1} from the output
    // buffer, which still holds x_{k-1}; none stores d.
    int fine_xstep = -1;
};
using ApplyArgs = ApplyArgsT<double>;

void launch_apply(int pro, int epi, const ApplyArgsT<double>& a, hipStream_t s);
void launch_apply(int pro, int epi, const ApplyArgsT<float>& a, hipStream_t s);
void launch_apply(int pro, int epi, const ApplyArgsT<float, bf16>& a,
                  hipStream_t s);
void configure_apply_kernels();  // LDS limits of every variant, once
// Finest-level Chebyshev step (plain prologue, launch_apply(PRO_PLAIN,
// EPI_CHEB) arithmetic): the tiled kernel of k_fine.hip when the level
// qualifies (uniform bands of even radius <= 16 after padding, five-point
// stencil, whole 64 x 16 tiles, 16-byte aligned vectors), else the general
// kernel.
void launch_smooth_fine(const ApplyArgsT<double>& a, hipStream_t s);
void launch_smooth_fine(const ApplyArgsT<float>& a, hipStream_t s);
void launch_smooth_fine(const ApplyArgsT<float, bf16>& a, hipStream_t s);
// false when the level does not qualify (nothing launched)
bool launch_smooth_fine_tiled(const ApplyArgsT<double>& a, hipStream_t s);
bool launch_smooth_fine_tiled(const ApplyArgsT<float>& a, hipStream_t s);
bool launch_smooth_fine_tiled(const ApplyArgsT<float, bf16>& a, hipStream_t s);

// ---- setup kernels (k_setup.hip) ------------------------------------
void launch_blur_band(const double* taps, int r, int n, int bc, double* band,
                      hipStream_t s);
void launch_transpose_band(const double* band, int n, int bw, int periodic,
                           double* out, hipStream_t s);
void launch_gram_band(const double* aband, int n, int ra, int periodic,
                      double* gband, int bwg, hipStream_t s);
void launch_galerkin_band(const double* fband, int nf, int bwf, int periodic,
                          double* cband, int bwc, hipStream_t s);
void launch_band_stats(const double* band, int n, int bw, double* diag,
                       double* rowabs, hipStream_t s);
void launch_fine_stencil(const double* d, int nv, int nh, int periodic,
                         double* planes, hipStream_t s);
void launch_galerkin_stencil(const double* fplanes, int nvf, int nhf,
                             int periodic, double* cplanes, hipStream_t s);
void launch_stencil_rowabs(const double* planes, int nv, int nh, int periodic,
                           double* rowabs, hipStream_t s);
void launch_gershgorin(const LevelGeom& g, const double* lam2, int nslot,
                       double* rho, hipStream_t s);
void launch_cheb_coeffs(const double* rho, int nslot, double ratio, int nu,
                        int stride, double* cheb, hipStream_t s);
void launch_coarse_assemble(const LevelGeom& g, const double* lam2, int nslot,
                            double* Kc, hipStream_t s);
void launch_cholesky_inverse(double* Kc, int n, int nslot, double* work,
                             int* info, hipStream_t s);
void launch_check_weights(const double* d, int64_t n, int* bad,
                          hipStream_t s);

// ---- PCG kernels (k_pcg.hip) ------------------------------------------

int vec_blocks(int64_t n);  // partial-sum slots per vector
void launch_broadcast(const double* src, int64_t n, int nslot, double* dst,
                      hipStream_t s);
void launch_axpy_sub(const double* f, int f_shared, const double* kx,
                     int64_t n, int nslot, double* r, hipStream_t s);
void launch_dot(const double* a, const double* b, int64_t n, int nslot,
                const int* slots, const int* active, double* part,
                hipStream_t s);
void launch_update_xr(SlotState* st, int* active, const int* slots,
                      int64_t n, int nslot, double* x, double* r,
                      const double* p, const double* q, const double* part_pq,
                      int npq, int parity, double* part_rr, hipStream_t s);
void launch_pcg_init(SlotState* st, int nslot, const double* fparts, int nf,
                     const double* rparts, int nr, double tol, int absolute,
                     int maxit, int* active, hipStream_t s);
void launch_sumsq_slots(const double* a, int64_t n, int nslot, double* part,
                        hipStream_t s);
void launch_reduce_slots(const double* part, int nparts, int nslot,
                         double* out, hipStream_t s);
void launch_weighted_grad_sq(const double* x, const double* d, int nv, int nh,
                             int periodic, int nslot, double* part,
                             hipStream_t s);
void launch_sub_sumsq(const double* a, const double* b, int64_t n, int nslot,
                      double* part, hipStream_t s);

// ---- sparse operators (k_csr.hip, k_ct.hip) ------------------------------
void launch_scan_excl(const int64_t* cnt, int64_t n, int64_t* out,
                      hipStream_t s);
void launch_csr_transpose_count(const int* ci, int64_t nnz,
                                unsigned long long* cnt, hipStream_t s);
void launch_csr_transpose_fill(const int64_t* rp, const int* ci,
                               const double* va, int64_t m, int64_t n,
                               const int64_t* rpt, unsigned long long* cursor,
                               int* cit, double* vat, int* err, hipStream_t s);
void launch_csr_coarsen(const int64_t* rp, const int* ci, const double* va,
                        int64_t m, int nvf, int nhf, int periodic, int mode,
                        int64_t* cnt, const int64_t* rpc, int* cic,
                        double* vac, int* err, hipStream_t s);
void launch_row_sumsq(const int64_t* rpt, const double* vat, int64_t n,
                      double* out, hipStream_t s);
template <class VT, class XT, class YT>
void launch_spmv(const int64_t* rp, const int* ci, const VT* va, int64_t nrows,
                 int64_t xstride, const XT* x, int x_shared, int64_t ystride,
                 YT* y, int nslot, const int* slots, const int* active,
                 hipStream_t s);
void launch_dense_gram(const int64_t* rpt, const int* cit, const double* vat,
                       int nc, double* G, hipStream_t s);
void launch_f64_from_f32(const float* a, int64_t n, double* b, hipStream_t s);
void launch_ct_apply(int pro, int epi, const ApplyArgsT<double>& a,
                     hipStream_t s);
void launch_ct_apply(int pro, int epi, const ApplyArgsT<float>& a,
                     hipStream_t s);
int ct_parts(int64_t n);   // partial sums per slot of a sparse-level kernel
void launch_gershgorin_ct(const LevelGeom& g, const double* lam2, int nslot,
                          double* rho, hipStream_t s);
void launch_coarse_assemble_ct(const LevelGeom& g, const double* G,
                               const double* lam2, int nslot, double* Kc,
                               hipStream_t s);

// FP32 V-cycle boundary (k_pcg.hip)
void launch_to_f32(const double* src, int64_t n, int nslot, const int* slots,
                   float* dst, hipStream_t s);
// Boundary of a reduced-precision V-cycle (V = float or bf16): narrowing of
// r (after the convergence test when st is given), widening of z with the
// partials of r . z (and z . q).
template <class V>
void launch_vc_enter(SlotState* st, int* active, const int* slots, int nslot,
                     const double* part_rr, int nrr, int64_t n, const double* r,
                     V* rlo, hipStream_t s);
template <class V>
void launch_vc_exit(const int* slots, const int* active, int nslot, int64_t n,
                    int npart, const V* zlo, double* z, const double* r,
                    const double* q, double* part_rz, double* part_zq,
                    hipStream_t s);

int apply_tiles(const LevelGeom& g);

// ---- coarse tail (k_tail.hip) -----------------------------------------
constexpr int TAIL_MAX_POINTS = 1024;   // levels this small run in the tail
constexpr int TAIL_MAX_LEVELS = 8;

struct TailLevel {
    int nv = 0, nh = 0;
    BandDev gv, gh;                  // band tables are always present
    StencilDev S;
    const double* cheb = nullptr;    // per slot Chebyshev (c1, c2) pairs
    int nu = 2;                      // smoothing steps on this level
};

// The tail computes in FP64; IO is the type of its right-hand side and
// result (float under the FP32 V-cycle).
template <class IO>
struct TailArgsT {
    int nlev = 0;                    // tail levels, the last is the coarsest
    TailLevel lev[TAIL_MAX_LEVELS];
    int cheb_stride = 0, periodic = 0;
    const double* lam2 = nullptr;
    const int* slots = nullptr;
    const int* active = nullptr;
    const IO* f = nullptr;           // right-hand side on the first tail level
    IO* z = nullptr;                 // result on the first tail level
    const double* W = nullptr;       // coarsest W = L^{-1} and W^T per slot
    int dot = 0;                     // write partials of f . z (level 0)
    double* part = nullptr;
    int part_stride = 0;
    int gate = 0;                    // convergence test first (level 0)
    SlotState* st = nullptr;
    int* active_w = nullptr;
    const double* part_rr = nullptr;
    int nrr = 0;
};

using TailArgs = TailArgsT<double>;

void launch_tail(const TailArgsT<double>& a, int nslot, hipStream_t s);
void launch_tail(const TailArgsT<float>& a, int nslot, hipStream_t s);
void launch_tail(const TailArgsT<bf16>& a, int nslot, hipStream_t s);
template <class IO>
size_t tail_lds_bytes(const TailArgsT<IO>& a);
size_t apply_lds_bytes(const LevelGeom& g, int epi);
size_t apply_lds_bytes(const LevelGeomT<float>& g, int epi);

}  // namespace rls
