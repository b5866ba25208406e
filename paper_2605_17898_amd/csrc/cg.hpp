// CG driver interface (see cg.hip).
#pragma once

#include "internal.hpp"
#include "vec.hpp"

namespace mfgp {

struct CgBufs {
    float* R = nullptr;
    float* P = nullptr;
    float* AP = nullptr;
    double* R64 = nullptr;
    double* scal = nullptr;   // [8][t]
    int* ints = nullptr;      // [6][t]
    double* dots = nullptr;
    double* resid = nullptr;
    float* apply = nullptr;
    void* sum = nullptr;      // sum_scratch_bytes(n, t): the terms of a kernel sum
    void* gram = nullptr;     // gram_prep_bytes(n) for n >= kGramMinN: the Gram data of the points,
                              // prepared once per solve (null below kGramMinN)
};

CgBufs carve_cg(Carver& cv, int64_t n, int t, int precision);
// The CG vectors only (no product or residual scratch): for operators that
// bring their own (structured kernel interpolation).
CgBufs carve_cg_vectors(Carver& cv, int64_t n, int t);

// Runs CG on K_y X = B (op prescaled, U filled).  Returns the worst column status.
int cg_run(const Operator& op, const float* B, int t, double* X, const mfgp_cg_opts& o,
           mfgp_cg_info* info, double* coeff, int max_iter, const CgBufs& b, hipStream_t s);

struct Precond;
// Extra buffers of the preconditioned solver: z = P^{-1} r and the Woodbury scratch.
struct PcgBufs {
    float* Zv = nullptr;       // [n, t]
    double* pc = nullptr;      // pc_scratch_doubles(n, k, t)
    double* rz0 = nullptr;     // [t] b^T P^{-1} b of the first cycle
};
PcgBufs carve_pcg(Carver& cv, int64_t n, int k, int t);
// Preconditioned CG (x0 = 0) with the same stopping rule, FP64 solution and
// refinement as cg_run; logs the (alpha, beta) of the first cycle, which give
// the Lanczos tridiagonal of P^{-1/2} K_y P^{-1/2}.
int pcg_run(const Operator& op, const Precond& pc, const float* B, int t, double* X, const mfgp_cg_opts& o,
            mfgp_cg_info* info, double* coeff, int max_iter, const CgBufs& b, const PcgBufs& pb, hipStream_t s);

}  // namespace mfgp
