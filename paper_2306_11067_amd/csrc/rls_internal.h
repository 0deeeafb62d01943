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

// A banded n x n operator along one image axis.  Row r, offset k in
// [-bw, bw] is the coefficient of x(map(r + k)).  `uniform` rows all equal
// `taps` (the index map supplies the boundary); otherwise `table` holds
// every row, with zeros where r + k falls outside a non-wrapping axis.
struct BandDev {
    int n = 0;
    int bw = 0;
    int map = MAP_ZERO;
    int uniform = 0;
    const double* taps = nullptr;   // 2bw+1
    const double* table = nullptr;  // n * (2bw+1)
    const double* diag = nullptr;   // n
    const double* rowabs = nullptr; // n: sum_k |row r|
};

// Galerkin stencil of L^T D^2 L on one level, five planes of n values:
// c (centre), cn (i+1, j), ce (i, j+1), cne (i+1, j+1), cse (i-1, j+1).
struct StencilDev {
    const double* c = nullptr;
    const double* cn = nullptr;
    const double* ce = nullptr;
    const double* cne = nullptr;
    const double* cse = nullptr;
    const double* rowabs = nullptr;  // sum_j |S_ij|
    int nine = 0;                    // 0: cne/cse are identically zero
    int periodic = 0;
};

struct LevelGeom {
    int nv = 0, nh = 0;
    BandDev gv, gh;                  // separable Gram G_h (x) G_v
    StencilDev S;
};

// Tile of the level-operator kernel (i is the contiguous axis).
constexpr int TILE_Y = 64;
constexpr int TILE_X = 16;
constexpr int APPLY_THREADS = 256;

// Prologue: how the operand v of K v is formed while loading a tile.
enum Prologue : int {
    PRO_PLAIN = 0,   // v = in
    PRO_PUPDATE = 1  // v = z + beta * p_old ; p_new = v (interior)
};
// Epilogue: what is done with (v, K v) at each output point.
enum Epilogue : int {
    EPI_STORE = 0,   // out = K v
    EPI_DOT = 1,     // out = K v ; partial sum of v . K v
    EPI_RESID = 2,   // out = f - K v
    EPI_CHEB = 3     // res = f - K v ; d = c1 d + c2 res / diag ; out = v + d
};

struct ApplyArgs {
    LevelGeom g;
    int nslot = 0;
    const double* lam2 = nullptr;    // per slot lambda^2
    const int* active = nullptr;     // per slot, may be null (all active)
    const double* in = nullptr;      // v (or z for PRO_PUPDATE), slot stride n
    const double* pold = nullptr;    // PRO_PUPDATE
    double* pnew = nullptr;          // PRO_PUPDATE
    const double* beta = nullptr;    // PRO_PUPDATE, per slot
    double* out = nullptr;
    const double* f = nullptr;       // EPI_RESID / EPI_CHEB right-hand side
    int f_shared = 0;                // f has one vector for all slots
    double* d = nullptr;             // EPI_CHEB direction, in place
    const double* cheb = nullptr;    // EPI_CHEB per slot (c1, c2) pairs
    int cheb_stride = 0;             // doubles between slots in cheb
    double* part = nullptr;          // EPI_DOT partials [slot][tile]
};

void launch_apply(int pro, int epi, const ApplyArgs& a, hipStream_t s);

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
                        double* cheb, hipStream_t s);
void launch_coarse_assemble(const LevelGeom& g, const double* lam2, int nslot,
                            double* Kc, hipStream_t s);
void launch_cholesky_inverse(double* Kc, int n, int nslot, double* work,
                             int* info, hipStream_t s);
void launch_check_weights(const double* d, int64_t n, int* bad,
                          hipStream_t s);

// ---- vector / multigrid kernels (k_vec.hip) -------------------------
void launch_jacobi_init(const LevelGeom& g, int nslot, const double* lam2,
                        const int* active, const double* f, int f_shared,
                        const double* cheb, int cheb_stride, double* x,
                        double* d, hipStream_t s);
void launch_restrict(const LevelGeom& fine, const LevelGeom& coarse, int nslot,
                     const int* active, const double* res, double* fc,
                     hipStream_t s);
void launch_prolong_add(const LevelGeom& fine, const LevelGeom& coarse,
                        int nslot, const int* active, const double* ec,
                        double* x, hipStream_t s);
void launch_coarse_solve(const double* Kinv, int n, int nslot,
                         const int* active, const double* f, double* z,
                         hipStream_t s);

// ---- PCG kernels (k_pcg.hip) ------------------------------------------
struct SlotState {
    double gamma;   // r . z
    double alpha;
    double beta;
    double rr;      // ||r||^2
    double target;  // residual norm target
    double fnorm;   // ||A^T b||
    int it;
    int active;
    int flags;
    int maxit;
};

int vec_blocks(int64_t n);  // partial-sum slots per vector
void launch_broadcast(const double* src, int64_t n, int nslot, double* dst,
                      hipStream_t s);
void launch_axpy_sub(const double* f, int f_shared, const double* kx,
                     int64_t n, int nslot, double* r, hipStream_t s);
void launch_dot(const double* a, const double* b, int64_t n, int nslot,
                const int* active, double* part, hipStream_t s);
void launch_update_xr(const SlotState* st, int64_t n, int nslot, double* x,
                      double* r, const double* p, const double* q,
                      double* part, hipStream_t s);
void launch_pcg_init(SlotState* st, int nslot, const double* fparts, int nf,
                     const double* rparts, int nr, const double* gparts,
                     int ng, double tol, int absolute, int maxit, int* active,
                     hipStream_t s);
void launch_finalize_alpha(SlotState* st, int nslot, const double* part,
                           int nparts, int* active, hipStream_t s);
void launch_finalize_rr(SlotState* st, int nslot, const double* part,
                        int nparts, int* active, hipStream_t s);
void launch_finalize_beta(SlotState* st, int nslot, const double* part,
                          int nparts, double* beta, int* active,
                          hipStream_t s);
void launch_sumsq_slots(const double* a, int64_t n, int nslot, double* part,
                        hipStream_t s);
void launch_reduce_slots(const double* part, int nparts, int nslot,
                         double* out, hipStream_t s);
void launch_weighted_grad_sq(const double* x, const double* d, int nv, int nh,
                             int periodic, int nslot, double* part,
                             hipStream_t s);
void launch_sub_sumsq(const double* a, const double* b, int64_t n, int nslot,
                      double* part, hipStream_t s);

int apply_tiles(const LevelGeom& g);

}  // namespace rls
