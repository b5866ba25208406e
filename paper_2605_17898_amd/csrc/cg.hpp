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
};

CgBufs carve_cg(Carver& cv, int64_t n, int t, int precision);

// Runs CG on K_y X = B (op prescaled, U filled).  Returns the worst column status.
int cg_run(const Operator& op, const float* B, int t, double* X, const mfgp_cg_opts& o,
           mfgp_cg_info* info, double* coeff, int max_iter, const CgBufs& b, hipStream_t s);

}  // namespace mfgp
