/*
 * rls.h -- batched lambda-sweep solver for regularized least squares on
 * AMD Instinct MI355X (gfx950).
 *
 * The library solves, for every regularization parameter lambda_i of a sweep,
 *
 *     (A^T A + lambda_i^2 L^T D^2 L) x_i = A^T b                      (1)
 *
 * the normal equations of min ||A x - b||^2 + lambda^2 ||D L x||^2 (paper:
 * Bolten, MacLachlan, Kilmer, "Multigrid preconditioning for regularized
 * least-squares problems", Section 1 eqs. (LSreg), (ml) and Section 3.2 eq.
 * (normal)).  L is the forward-difference gradient of Section 2 eq.
 * (gradient), D a nonnegative diagonal weighting of its rows (Section 2,
 * eq. (g) and the update D^(l) = diag(d^(l)) D^(l-1)).  All lambdas of a
 * sweep run together on the GPU with preconditioned conjugate gradients; the
 * preconditioner is one multigrid V-cycle (Algorithm 1) on a hierarchy that
 * does not depend on lambda (Section 3.2), so it is built once per weighting
 * and reused by every lambda.  Each solve returns x_i and the L-curve pair
 * (||A x_i - b||_2, ||D L x_i||_2) of Section 1.
 *
 * Layout.  An image of nv x nh pixels is a vector of n = nv*nh values,
 * pixel (i, j) at index i + nv*j (column-major, i vertical; Section 2).
 * A batch of vectors is stored vector after vector.  The weights d cover the
 * two gradient planes: d[i + nv*j] weights the vertical difference
 * x(i+1,j) - x(i,j), d[n + i + nv*j] the horizontal difference
 * x(i,j+1) - x(i,j).  With a Neumann gradient the last difference in each
 * direction is identically zero and its weight is ignored; with a periodic
 * gradient it wraps around.
 *
 * Memory.  "device" arguments are GPU pointers (for example torch tensor
 * data_ptr() values) on the device current at rls_setup; "host" arguments are
 * CPU pointers.  The caller owns every pointer it passes; the library copies
 * what it keeps.  All device work is ordered on the caller's stream (a
 * hipStream_t passed as void*, NULL for the null stream); every call returns
 * after its results are in place (host outputs written, device outputs
 * complete on that stream).
 *
 * Errors.  Calls never throw; they return an rls_status and leave a message
 * for rls_last_error() (thread-local).  Per-lambda non-convergence or
 * breakdown is reported in rls_solve_info.flags, not as a call failure.
 */
#ifndef RLS_H
#define RLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int rls_status;
#define RLS_OK             0
#define RLS_E_ARG         -1   /* invalid argument (sizes, values, nulls)   */
#define RLS_E_HIP         -2   /* a HIP runtime call failed                 */
#define RLS_E_OOM         -3   /* device allocation failed                  */
#define RLS_E_NOT_SPD     -4   /* non-positive pivot in a coarsest solve    */
#define RLS_E_UNSUPPORTED -5   /* valid but not supported configuration     */
#define RLS_E_STATE       -6   /* call out of order / bad handle            */

/* Forward operator kinds. */
#define RLS_OP_BLUR_SEPARABLE 1  /* A = A_h (x) A_v, 1D convolutions        */
#define RLS_OP_CSR            2  /* A general sparse m x n (tomography)      */

/* Boundary conditions of a separable blur: (A_v x)_i = sum_k t_k x(i-k),
 * k = -r..r, with x outside [0, n) taken from the periodic continuation,
 * the half-sample symmetric reflection (x(-1) = x(0)), or zero. */
#define RLS_BC_PERIODIC   0
#define RLS_BC_REFLECTIVE 1
#define RLS_BC_ZERO       2

/* Gradient boundary (also selects the multigrid transfer boundary). */
#define RLS_L_NEUMANN  0
#define RLS_L_PERIODIC 1

/* Arithmetic of the iteration.  FP64: everything in double precision.
 * MIXED_FP32: the PCG iteration (x, r, p, q, all dot products, the
 * convergence test and the final residual) stays FP64; the V-cycle
 * preconditioner (level vectors, Gram bands, Galerkin stencils and their
 * arithmetic) runs in FP32, except the coarse tail levels and the coarsest
 * Cholesky solve, which stay FP64.  An FP32 V-cycle is not exactly the same
 * linear map at every application, so PCG then uses the flexible
 * (Polak-Ribiere) beta; the attainable accuracy is that of the FP64
 * residual (Sec. 3, Algorithm 1 as the preconditioner of CG).
 * MIXED_BF16: as MIXED_FP32, with the V-cycle's level vectors stored in
 * BF16 (round to nearest even on every store; bands, stencils and all
 * arithmetic FP32, coarse tail FP64).  Blur operators only. */
#define RLS_PREC_FP64       0
#define RLS_PREC_MIXED_FP32 1
#define RLS_PREC_MIXED_BF16 2

/* Tolerance semantics of rls_solve_sweep. */
#define RLS_TOL_RELATIVE 0   /* ||A^T b - K x_i|| <= tol * ||A^T b||      */
#define RLS_TOL_ABSOLUTE 1   /* ||A^T b - K x_i|| <= tol (paper Sec. 3.3) */

/* Per-lambda result flags. */
#define RLS_FLAG_CONVERGED 1
#define RLS_FLAG_MAXIT     2
#define RLS_FLAG_BREAKDOWN 4   /* p^T K p <= 0 or r^T z <= 0                */
#define RLS_FLAG_NONFINITE 8

typedef struct {
    int kind;               /* RLS_OP_BLUR_SEPARABLE or RLS_OP_CSR           */
    /* separable blur (paper Section 4.6: A is a Kronecker product of 1D
     * Toeplitz-type matrices) */
    int bc;                 /* RLS_BC_*                                      */
    int r_v, r_h;           /* tap radii: 2r+1 taps per direction            */
    const double* taps_v;   /* host, 2*r_v+1 values, t_{-r}..t_{r}           */
    const double* taps_h;   /* host, 2*r_h+1 values                          */
    /* general sparse A (RLS_OP_CSR, e.g. a tomography projector): m rows
     * over the n = nv*nh pixels, rows sorted by column, values >= 0; runs
     * with RLS_PREC_MIXED_FP32 only; at most 512 nonzeros per row and 4096
     * per column (the on-GPU hierarchy build) */
    int64_t m, nnz;
    const int64_t* rowptr;  /* host, m+1 */
    const int32_t* col;     /* host, nnz */
    const float* val;       /* host, nnz */
} rls_op_desc;

typedef struct {
    int nv, nh;             /* image size; both divisible by 2^(levels-1)    */
    int lbc;                /* RLS_L_NEUMANN or RLS_L_PERIODIC               */
    int levels;             /* multigrid levels >= 1; the coarsest level is
                               solved exactly (Algorithm 1), at most 1024
                               unknowns, every level at least 4 x 4          */
    int nu;                 /* Chebyshev smoothing steps before and after the
                               coarse correction on the finest level
                               (V(nu,nu)), 1..256                            */
    double cheb_ratio;      /* finest-level smoothing interval
                               [rho/ratio, rho], rho the Gershgorin bound of
                               diag(K_k)^-1 K_k; > 1                         */
    int precision;          /* RLS_PREC_FP64, _MIXED_FP32 or _MIXED_BF16     */
    int nu_coarse;          /* same on the coarser levels (0: = nu), 1..256 */
    double cheb_ratio_coarse; /* same on the coarser levels (0: = cheb_ratio) */
} rls_grid_desc;

typedef struct {
    int maxit;              /* PCG iteration cap per lambda (>= 1)           */
    int tol_mode;           /* RLS_TOL_RELATIVE / RLS_TOL_ABSOLUTE           */
    int poll_every;         /* host convergence check period, iterations     */
    int graph;              /* 1: replay iteration chunks as HIP graphs;
                               0: launch kernels one by one (same results)   */
} rls_sweep_opts;

typedef struct {
    int iters;              /* PCG iterations (products K p) taken           */
    int flags;              /* RLS_FLAG_*                                    */
    double relres;          /* recursive ||r|| / ||A^T b|| at exit           */
    double relres_true;     /* ||A^T b - K x|| / ||A^T b|| recomputed        */
} rls_solve_info;

typedef struct rls_problem rls_problem;

/* Build a problem: copy the operator description, construct the lambda-free
 * multigrid hierarchy (separable Gram bands of A_k^T A_k = P^T A^T A P for
 * the blur, paper Section 3.2 one-sided hierarchy) and install the weights.
 * d: device, 2n values >= 0 and finite, or NULL for D = I (paper D^(0) = I).
 * On success *out receives a handle to free with rls_destroy.
 * Kernel choice: the finest-level Chebyshev step of a blur problem takes a
 * tiled kernel specialised for the band radius when the grid is a whole
 * number of 64 x 16 tiles and the Gram bands are uniform (periodic, or
 * reflective with a symmetric PSF); the environment variable
 * RLS_FINE_KERNEL=generic, read here, makes this problem use the general
 * level-operator kernel instead (same arithmetic up to rounding).
 * Errors: RLS_E_ARG (bad sizes, radii >= n/2, non-finite taps, nu/levels out
 * of range), RLS_E_UNSUPPORTED (precision, boundary pair, a sparse
 * operator with a precision other than RLS_PREC_MIXED_FP32 or rows or
 * columns beyond the limits above, a blur band wider than a level or its
 * LDS tile), RLS_E_OOM,
 * RLS_E_HIP. */
rls_status rls_setup(rls_problem** out, const rls_op_desc* A,
                     const rls_grid_desc* g, const double* d, void* stream);

/* Install the weights of a new outer iteration l: rebuild the Galerkin
 * coarse stencils of L^T D^2 L (paper Section 3.2: formed once per
 * weighting, reused for every lambda).  d: device, 2n values (NULL: D = I).
 * Errors: RLS_E_STATE (null handle), RLS_E_ARG (negative or non-finite
 * weight), RLS_E_HIP. */
rls_status rls_set_weights(rls_problem* p, const double* d, void* stream);

/* Solve (1) for lam[0..nlam-1] at once.
 * b:        device, n values (the data; A is square for the blur).
 * lam:      host, nlam values > 0.
 * tol:      > 0, see opts->tol_mode (NULL opts: relative, maxit 100000,
 *           poll every 32 iterations, graphs on).
 * x0:       device, nlam*n initial guesses, or NULL for zero.
 * x:        device, nlam*n solutions (may alias x0).
 * resnorm:  host, nlam values ||A x_i - b||_2 (may be NULL).
 * seminorm: host, nlam values ||D L x_i||_2 (may be NULL).
 * info:     host, nlam records (may be NULL).
 * Errors: RLS_E_ARG (nlam < 1, lam <= 0 or non-finite, tol <= 0, null
 * b / x), RLS_E_NOT_SPD (coarsest matrix not positive definite),
 * RLS_E_OOM, RLS_E_HIP. */
rls_status rls_solve_sweep(rls_problem* p, const double* b, const double* lam,
                           int nlam, double tol, const rls_sweep_opts* opts,
                           const double* x0, double* x, double* resnorm,
                           double* seminorm, rls_solve_info* info,
                           void* stream);

/* One sweep of a batch: the arguments of rls_solve_sweep for one problem,
 * and its outcome. */
typedef struct {
    rls_problem* prob;          /* distinct handle per entry                 */
    const double* b;            /* as in rls_solve_sweep                     */
    const double* lam;
    int nlam;
    double tol;
    const rls_sweep_opts* opts;
    const double* x0;
    double* x;
    double* resnorm;
    double* seminorm;
    rls_solve_info* info;
    rls_status status;          /* out: this sweep's status                  */
} rls_sweep;

/* Solve the sweeps of several problems of uneven sizes together (the
 * lambda sweeps of the paper's Section 4 experiments, one per problem and
 * outer weighting).  Each problem runs on a stream of its own, driven by a
 * host thread of its own, so the small problems' latency-bound launches
 * overlap on the GPU; every problem's results are bitwise those of
 * rls_solve_sweep on it alone.  The problems' work is ordered after the
 * work already on `stream`, and the call returns when every sweep has
 * finished.  Returns the first failing entry's status (each entry's own
 * status is in sweeps[i].status).
 * Errors: RLS_E_ARG (nsweep < 1, null sweeps or handle, a handle listed
 * twice), otherwise those of rls_solve_sweep. */
rls_status rls_solve_batch(rls_sweep* sweeps, int nsweep, void* stream);

/* Free a handle (NULL is ignored). */
void rls_destroy(rls_problem* p);

/* Message of the last failed call on this thread ("" if none). */
const char* rls_last_error(void);

/* ---------------------------------------------------------------------
 * Step-level entry points.  Each runs one step of the solver on its own,
 * with the same kernels rls_solve_sweep uses, so that every step can be
 * checked in isolation.  Level 0 is the finest grid.
 * ------------------------------------------------------------------- */

/* Grid size of a level. Errors: RLS_E_STATE, RLS_E_ARG (level range). */
rls_status rls_level_shape(const rls_problem* p, int level, int* nv, int* nh);

/* out_i = K_level(lam_i) v_i for i < nlam, K_level = P^T ... K ... P the
 * Galerkin level operator (paper Section 3.2).  v, out: device,
 * nlam * n_level values.  lam: host. */
rls_status rls_apply_normal(rls_problem* p, int level, const double* lam,
                            int nlam, const double* v, double* out,
                            void* stream);

/* z_i = V-cycle(lam_i) applied to r_i (Algorithm 1 with gamma = 1, the
 * preconditioner of rls_solve_sweep).  r, z: device, nlam * n values. */
rls_status rls_vcycle(rls_problem* p, const double* lam, int nlam,
                      const double* r, double* z, void* stream);

/* Copy the Galerkin stencil of L^T D^2 L on a level to the host: five
 * planes of n_level values: centre, coupling to (i+1,j), to (i,j+1), to
 * (i+1,j+1) and to (i-1,j+1) (the other four follow by symmetry). */
rls_status rls_get_stencil(const rls_problem* p, int level, double* out);

/* Copy one direction (0 vertical, 1 horizontal) of the separable Gram
 * A_k^T A_k = G_h (x) G_v on a level to the host as a band: *bw receives
 * the half bandwidth; out (host, may be NULL to query bw) receives
 * n_dir * (2 bw + 1) values, row r, offset k in [-bw, bw] at
 * out[r*(2bw+1) + k + bw] (coefficient of x(r+k), wrapped if periodic). */
rls_status rls_get_gram_band(const rls_problem* p, int level, int dir,
                             int* bw, double* out);

/* Gershgorin bounds rho_k(lam_i) of diag(K_k)^-1 K_k used for the
 * Chebyshev interval: rho (host) receives nlam values. */
rls_status rls_gershgorin(rls_problem* p, int level, const double* lam,
                          int nlam, double* rho, void* stream);

/* Live timing of the sweep's most frequent kernel: the finest-level level
 * operator with the Chebyshev-step epilogue and a plain prologue (all but
 * two of the 2 nu - 1 finest-level smoothing launches of a V-cycle).  While
 * enabled, rls_solve_sweep launches kernels one by one instead of replaying
 * graphs, and every run of consecutive such launches (the pre- and the
 * post-smoothing steps of a V-cycle) is bracketed by one pair of HIP events
 * on the launch stream.
 * rls_kernel_timer(p, 1) enables and resets, (p, 0) disables.
 * rls_kernel_timer_read returns the number of timed launches, their summed
 * duration in seconds and their summed algorithmic bytes: per pixel, 32
 * bytes per active lambda for the tiled kernel, which runs the three-term
 * form of the recurrence (read x_k, x_{k-1} or the first step's direction,
 * f; write x_{k+1}), or 40 for the general kernel (read x, f, d; write x,
 * d), plus, for launches with an active lambda, 16 bytes of shared stencil
 * couplings (north and east; the centre is minus the sum of the four
 * couplings), every array counted once. */
rls_status rls_kernel_timer(rls_problem* p, int enable);
rls_status rls_kernel_timer_read(const rls_problem* p, long long* launches,
                                 double* seconds, double* bytes);

/* y = A x (forward blur) or x = A^T y for nvec vectors (device). */
rls_status rls_apply_forward(rls_problem* p, const double* x, double* y,
                             int nvec, void* stream);
rls_status rls_apply_adjoint(rls_problem* p, const double* y, double* x,
                             int nvec, void* stream);

/* ---------------------------------------------------------------------
 * Outer reweighting loop (paper Algorithm 2, Section 3.6).
 * ------------------------------------------------------------------- */

/* Weight update of eq. (g) (paper Section 2) from a solution x (device, n
 * values): with w = |D L x| over the 2n gradient entries (L the forward
 * differences of the problem's gradient, D its current weights),
 * g = w / ||w||_inf and D <- diag(1 - g^q) D; then the per-weighting
 * set-up for the new D, as rls_set_weights does.  ||w||_inf = 0 leaves D
 * unchanged.  gmax: host, receives ||w||_inf (may be NULL).  Synchronous.
 * Errors: RLS_E_STATE, RLS_E_ARG (null x, q <= 0 or non-finite), RLS_E_OOM,
 * RLS_E_HIP. */
rls_status rls_update_weights(rls_problem* p, const double* x, double q,
                              double* gmax, void* stream);

/* Copy of the current weights D (2n values, vertical plane first) into d
 * (device); ones for D = I.  Errors: RLS_E_STATE, RLS_E_ARG, RLS_E_HIP. */
rls_status rls_get_weights(const rls_problem* p, double* d, void* stream);

/* L-curve corner (paper Section 1, the criterion of Hansen and O'Leary):
 * natural cubic splines of log10 rho and log10 eta over log10 lambda
 * through the m points, their curvature sampled 64 times per interval, and
 * *index = the point nearest, in the log-log plane, to the sample of
 * largest curvature.  lam, rho, eta: host, m values, positive and finite,
 * lam strictly increasing.  Host only, no GPU work.
 * Errors: RLS_E_ARG (m < 3, null pointers, values out of range). */
rls_status rls_lcurve_corner(const double* lam, const double* rho,
                             const double* eta, int m, int* index);

/* Pruned lambda range of paper Section 3.4 (0-based, inclusive): ten
 * indices from i_prev - 2 to i_prev + 7, shifted to the first or last ten
 * near the ends.  Errors: RLS_E_ARG (m < 10, i_prev out of range). */
rls_status rls_trim_window(int i_prev, int m, int* lo, int* hi);

/* Outcome of rls_regularize. */
typedef struct {
    int outer;          /* outer iterations run                              */
    int stopped;        /* 1: the stopping rule of Section 3.5 fired         */
    int chosen_index;   /* lambda index of the returned solution            */
    long long iters;    /* PCG iterations summed over all solves             */
} rls_outer_info;

/* Algorithm 2: starting from D = I, outer iteration l solves every lambda
 * (l = 1) or the pruned range around the previous choice (rls_trim_window)
 * with rls_solve_sweep, picks the corner lambda (rls_lcurve_corner), stops
 * once the same index was picked three times in a row (Section 3.5), and
 * otherwise updates D from the chosen solution (rls_update_weights).  Each
 * lambda's solve starts from that lambda's latest solution (zero at first).
 * b: device, the data.  lam: host, m >= 10 values, positive, strictly
 * increasing.  q > 0: the exponent of eq. (g).  tol, opts: as in
 * rls_solve_sweep.  chosen: host, maxouter ints, the index picked at each
 * outer iteration.  x: device, n values, the solution at the last pick.
 * The library allocates m n doubles of device memory for the solutions
 * while it runs; on return the problem holds the weights of the last
 * solve.  Synchronous.  Errors: RLS_E_STATE, RLS_E_ARG, and those of
 * rls_solve_sweep. */
rls_status rls_regularize(rls_problem* p, const double* b, const double* lam,
                          int m, double q, double tol,
                          const rls_sweep_opts* opts, int maxouter,
                          int* chosen, double* x, rls_outer_info* info,
                          void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RLS_H */
