// Outer reweighting loop (paper Algorithm 2): launches and host helpers
// shared by k_outer.hip and the C-ABI.
#pragma once
#include <hip/hip_runtime.h>

namespace rls {

constexpr int CORNER_SAMPLES = 64;   // curvature samples per lambda interval
constexpr int TRIM_SIZE = 10;        // lambdas in a pruned sweep

// New weights dout (2n) = (1 - (|D L x| / ||D L x||_inf)^q) * d, d = NULL
// meaning D = I; *top (device) receives ||D L x||_inf.  part: device
// scratch of weight_update_parts() doubles.
void launch_weight_update(const double* x, const double* d, int nv, int nh,
                          int periodic, double q, double* part, double* dout,
                          double* top, hipStream_t s);
int weight_update_parts();

// Index of the lambda closest to the L-curve's corner; m >= 3, lam strictly
// increasing, every value positive and finite (checked by the caller).
int lcurve_corner_host(const double* lam, const double* rho, const double* eta,
                       int m);

// Inclusive range of the pruned sweep around the previous choice; m >=
// TRIM_SIZE, 0 <= i_prev < m.
void trim_window_host(int i_prev, int m, int* lo, int* hi);

}  // namespace rls
