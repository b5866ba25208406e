// CG state and column-vector kernels (see vec.hip).
#pragma once

#include "common.hpp"

namespace mfgp {

// Device pointers of a CG run on [n, t] blocks.
struct CgState {
    double* x;        // [n, t] solution (FP64)
    float* r;         // [n, t] residual
    float* p;         // [n, t] search direction
    float* ap;        // [n, t] K_y p
    double* rr;       // [t] r^T r
    double* bnorm2;   // [t] b^T b
    double* pap;      // [t] p^T K_y p
    double* alpha;    // [t]
    double* beta;     // [t]
    double* rrn;      // [t] new r^T r (single-problem path)
    int* active;      // [t] 1 while the column iterates
    int* status;      // [t] mfgp_status
    int* iters;       // [t] iterations done
    int* lanlen;      // [t] logged Lanczos length
    double* coeff;    // [t][max_iter][2] (alpha, beta) log, may be null
};

int stripe_blocks(int64_t n, int t);
// st.pap = p^T (A p) per column and the step length alpha = st.rr / st.pap
// in two launches: the striped partial dots, then one block per column
// (breakdown when p^T A p is not positive and finite).
hipError_t cg_pap_alpha(const CgState& st, int64_t n, int t, double* scratch, hipStream_t s);
hipError_t cg_update_and_beta(const CgState& st, int64_t n, int t, double* scratch, double tol,
                              int log_coeffs, int max_iter, hipStream_t s);
// x += alpha p, r -= alpha A p for active columns; rr_out[c] = r_c^T r_c (FP64).
hipError_t cg_update_rr(const CgState& st, int64_t n, int t, double* scratch, double* rr_out, hipStream_t s);
hipError_t cg_restart(const CgState& st, const double* R64, int64_t n, int t, const int* restart,
                      hipStream_t s);
hipError_t cg_activate(const CgState& st, int t, const int* restart, const double* rr_new,
                       hipStream_t s);
hipError_t cg_replace(const CgState& st, const double* R64, int64_t n, int t, const int* flag,
                      double* scratch, double* rr_tmp, hipStream_t s);
hipError_t fill_f64(double* x, int64_t total, double v, hipStream_t s);
hipError_t copy2_f32(const float* src, float* a, float* b, int64_t total, hipStream_t s);
hipError_t f64_to_f32(const double* src, float* dst, int64_t total, hipStream_t s);
// Stochastic diagonal estimate of the predictive variance from probes Z and
// Q = K_*f K_y^{-1} K_f* Z ([m][p] each): var = s2 - sum_c Z Q / sum_c Z^2.
hipError_t diag_variance(const float* Z, const float* Q, int64_t m, int p, double s2, float* var, hipStream_t s);

}  // namespace mfgp
