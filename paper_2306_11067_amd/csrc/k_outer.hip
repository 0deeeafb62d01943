// Outer reweighting loop of Algorithm 2 (paper Section 3.6): the weight
// update of eq. (g) on the GPU, and the host-side choices between sweeps
// (L-curve corner, pruned lambda window).
//
// Weight update: with w = |D L x| over both gradient planes (vertical
// differences first, then horizontal, each plane indexed like the image),
//     g = w / ||w||_inf,   d = 1 - g^q,   D <- diag(d) D.
// Two passes over the 2n gradient entries, each on at most WMAX_BLOCKS
// grid-stride blocks: per-block maxima, then every block reduces the
// maxima itself and writes the new weights.  The maximum is exact, so the result does not depend on the
// launch shape.  ||w||_inf = 0 leaves D unchanged (g = 0).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "outer.h"

namespace rls {
namespace {

constexpr int WT = 256;            // threads per block
constexpr int WMAX_BLOCKS = 1024;  // most blocks of the maximum pass

// |d_e (L x)_e| for gradient entry e: forward difference along the
// contiguous axis (plane 0) or across it (plane 1); the last difference of
// a line is zero on a Neumann grid and wraps on a periodic one.
__device__ __forceinline__ double grad_entry(const double* __restrict__ x,
                                             const double* __restrict__ d,
                                             int nv, int nh, int periodic,
                                             int64_t e, int64_t n) {
    const int plane = e >= n;
    const int64_t k = e - (plane ? n : 0);
    const int i = (int)(k % nv), j = (int)(k / nv);
    double diff = 0.0;
    if (!plane) {
        if (i + 1 < nv) diff = x[k + 1] - x[k];
        else if (periodic) diff = x[k - (nv - 1)] - x[k];
    } else {
        if (j + 1 < nh) diff = x[k + nv] - x[k];
        else if (periodic) diff = x[i] - x[k];
    }
    const double v = d ? d[e] * diff : diff;
    return fabs(v);
}

__device__ __forceinline__ double block_max(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = WT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = fmax(red[t], red[t + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(WT)
k_weight_max(const double* __restrict__ x, const double* __restrict__ d,
             int nv, int nh, int periodic, double* __restrict__ part) {
    __shared__ double red[WT];
    const int64_t n = (int64_t)nv * nh, ne = 2 * n;
    double m = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * WT + threadIdx.x; e < ne;
         e += (int64_t)gridDim.x * WT)
        m = fmax(m, grad_entry(x, d, nv, nh, periodic, e, n));
    m = block_max(m, red);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void __launch_bounds__(WT)
k_weight_update(const double* __restrict__ x, const double* __restrict__ d,
                int nv, int nh, int periodic, double q,
                const double* __restrict__ part, int nparts,
                double* __restrict__ dout, double* __restrict__ top_out) {
    __shared__ double red[WT];
    double m = 0.0;
    for (int k = threadIdx.x; k < nparts; k += WT) m = fmax(m, part[k]);
    const double top = block_max(m, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) *top_out = top;
    const int64_t n = (int64_t)nv * nh, ne = 2 * n;
    for (int64_t e = (int64_t)blockIdx.x * WT + threadIdx.x; e < ne;
         e += (int64_t)gridDim.x * WT) {
        const double dp = d ? d[e] : 1.0;
        double dn = dp;
        if (top > 0.0) {
            const double g = grad_entry(x, d, nv, nh, periodic, e, n) / top;
            const double gq = q == 1.0 ? g : (q == 2.0 ? g * g : pow(g, q));
            dn = (1.0 - gq) * dp;
        }
        dout[e] = dn;
    }
}

// Natural cubic spline through (t_i, y_i): second derivatives M (M_0 =
// M_{m-1} = 0) from the tridiagonal continuity conditions.
void natural_spline(const std::vector<double>& t, const std::vector<double>& y,
                    std::vector<double>& M) {
    const int m = (int)t.size();
    M.assign(m, 0.0);
    if (m < 3) return;
    const int k = m - 2;
    std::vector<double> a(k), b(k), c(k), r(k);
    for (int i = 1; i <= k; ++i) {
        const double h0 = t[i] - t[i - 1], h1 = t[i + 1] - t[i];
        a[i - 1] = h0;
        b[i - 1] = 2.0 * (h0 + h1);
        c[i - 1] = h1;
        r[i - 1] = 6.0 * ((y[i + 1] - y[i]) / h1 - (y[i] - y[i - 1]) / h0);
    }
    for (int i = 1; i < k; ++i) {     // forward elimination
        const double w = a[i] / b[i - 1];
        b[i] -= w * c[i - 1];
        r[i] -= w * r[i - 1];
    }
    M[k] = r[k - 1] / b[k - 1];
    for (int i = k - 2; i >= 0; --i) M[i + 1] = (r[i] - c[i] * M[i + 2]) / b[i];
}

// Value, first and second derivative of the spline on [t_i, t_{i+1}] at
// offset s from t_i.
void spline_eval(const std::vector<double>& t, const std::vector<double>& y,
                 const std::vector<double>& M, int i, double s, double& v,
                 double& d1, double& d2) {
    const double h = t[i + 1] - t[i];
    const double b = (y[i + 1] - y[i]) / h - h * (2.0 * M[i] + M[i + 1]) / 6.0;
    const double c3 = (M[i + 1] - M[i]) / (6.0 * h);
    v = y[i] + s * (b + s * (0.5 * M[i] + s * c3));
    d1 = b + s * (M[i] + 3.0 * c3 * s);
    d2 = M[i] + 6.0 * c3 * s;
}

}  // namespace

void launch_weight_update(const double* x, const double* d, int nv, int nh,
                          int periodic, double q, double* part,
                          double* dout, double* top, hipStream_t s) {
    const int64_t ne = 2 * (int64_t)nv * nh;
    const int nb = (int)std::min<int64_t>((ne + WT - 1) / WT, WMAX_BLOCKS);
    hipLaunchKernelGGL(k_weight_max, dim3(nb), dim3(WT), 0, s, x, d, nv, nh,
                       periodic, part);
    // every block of the update pass reads the nb maxima first: the same
    // cap keeps that re-read small against the 40 bytes per entry it moves
    hipLaunchKernelGGL(k_weight_update, dim3(nb), dim3(WT), 0, s, x, d, nv, nh,
                       periodic, q, part, nb, dout, top);
}

int weight_update_parts() { return WMAX_BLOCKS; }

int lcurve_corner_host(const double* lam, const double* rho, const double* eta,
                       int m) {
    std::vector<double> t(m), X(m), Y(m), MX, MY;
    for (int i = 0; i < m; ++i) {
        t[i] = std::log10(lam[i]);
        X[i] = std::log10(rho[i]);
        Y[i] = std::log10(eta[i]);
    }
    natural_spline(t, X, MX);
    natural_spline(t, Y, MY);
    // the sample of largest curvature (first one on ties)
    double best = -INFINITY, bx = X[0], by = Y[0];
    for (int i = 0; i + 1 < m; ++i) {
        const double h = t[i + 1] - t[i];
        const int last = i + 2 == m;
        for (int k = 0; k < CORNER_SAMPLES + last; ++k) {
            const double s = k == CORNER_SAMPLES
                                 ? h
                                 : (t[i] + h * k / CORNER_SAMPLES) - t[i];
            double xv, x1, x2, yv, y1, y2;
            spline_eval(t, X, MX, i, s, xv, x1, x2);
            spline_eval(t, Y, MY, i, s, yv, y1, y2);
            const double kappa =
                (x1 * y2 - y1 * x2) / std::pow(x1 * x1 + y1 * y1, 1.5);
            if (kappa > best) { best = kappa; bx = xv; by = yv; }
        }
    }
    int idx = 0;
    double dmin = INFINITY;
    for (int i = 0; i < m; ++i) {
        const double dx = X[i] - bx, dy = Y[i] - by;
        const double dd = dx * dx + dy * dy;
        if (dd < dmin) { dmin = dd; idx = i; }
    }
    return idx;
}

void trim_window_host(int i_prev, int m, int* lo, int* hi) {
    *lo = std::max(std::min(i_prev - 2, m - TRIM_SIZE), 0);
    *hi = std::min(std::max(i_prev + TRIM_SIZE - 3, TRIM_SIZE - 1), m - 1);
}

}  // namespace rls
