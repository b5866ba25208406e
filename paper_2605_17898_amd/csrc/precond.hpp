// Rank-k pivoted-Cholesky preconditioner P = L L^T + sigma^2 I (see precond.hip).
#pragma once

#include "internal.hpp"

namespace mfgp {

// A built factor and its Woodbury data.  L is caller- or workspace-owned
// device memory, row q holding column q of the factor ([k][n], float32).
struct Precond {
    const float* L = nullptr;
    int k = 0;
    int64_t n = 0;
    double s2n = 0.0;       // sigma^2
    double logdet = 0.0;    // log|P|
    double* C = nullptr;    // device [k x k] column-major: lower Cholesky factor of S = s2n I + L^T L
    double* L64 = nullptr;  // device FP64 copy of L (column-major n x k)
};

// Device scratch (doubles) of pivoted_cholesky for n rows.
size_t pchol_scratch_doubles(int64_t n);
// Rank-k pivoted Cholesky of the noise-free s2 k(X, X) of the prescaled op:
// writes L [k][n] and the pivots piv [k] (device).  Columns past the numerical
// rank (remaining diagonal <= 1e-6 s2) are zero.
hipError_t pivoted_cholesky(const Operator& op, int k, float* L, int* piv, double* scratch, hipStream_t s);

// Device scratch (doubles) of the Woodbury data and one application to t columns.
size_t pc_scratch_doubles(int64_t n, int k, int t);
// Copies L to FP64, forms S = s2n I + L^T L (dgemm), factors it on the host
// (FP64), uploads C and sets logdet.  Synchronises the stream.  Returns hipErrorInvalidValue if S is not
// positive definite.
hipError_t pc_setup(Precond& pc, double* scratch, hipStream_t s);
// Z = P^{-1} R for [n, t] blocks (Woodbury, FP64 accumulation).
hipError_t pc_apply(const Precond& pc, const float* R, int t, float* Z, double* scratch, hipStream_t s);
// Z = L E + sqrt(s2n) G: probes z_c ~ N(0, P) from standard normal E [k][p], G [n][p].
hipError_t pc_probes(const float* L, int k, int64_t n, double s2n, const float* E, const float* G, int p,
                     float* Z, hipStream_t s);

}  // namespace mfgp
