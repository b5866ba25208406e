// Shared device helpers and internal launcher declarations for the mfgp library.
//
// Kernel entries are generated in FP32 from prescaled coordinates
//   u_i = x_i * c_f / l        (per dimension, done once per call)
// so that the per-entry work is a sum of squared differences followed by one
// hardware exp2 (v_exp_f32):
//   RBF          c = sqrt(log2(e) / 2):  k^ = 2^(-|u_i - u_j|^2)      = exp(-r^2/2)
//   Matern-nu    c = sqrt(2 nu) log2(e): q = |u_i - u_j|, k^ = P(q) 2^(-q),
//                with sqrt(2 nu) rho = q ln2 and P the Matern polynomial
// (the families of LightGP Sec. 3 "Kernels").  Every path computes an entry
// with the same instruction sequence (kentry below), so the FP32 operator
// the solver applies is one fixed matrix.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "../../include/mfgp.h"

namespace mfgp {

constexpr float kLn2 = 0.693147180559945309f;
constexpr float kLn2Sq3 = 0.160151004639400475f;  // ln(2)^2 / 3

// ---------------------------------------------------------------- entries

// Unit-outputscale kernel entry from the squared prescaled distance d2.
template <int FAM>
__device__ __forceinline__ float kentry(float d2) {
    if constexpr (FAM == MFGP_RBF) {
        return __builtin_amdgcn_exp2f(-d2);
    } else {
        const float q = __builtin_amdgcn_sqrtf(d2);
        const float e = __builtin_amdgcn_exp2f(-q);
        if constexpr (FAM == MFGP_MATERN12) {
            return e;
        } else if constexpr (FAM == MFGP_MATERN32) {
            return fmaf(q, kLn2, 1.0f) * e;
        } else {
            return fmaf(fmaf(q, kLn2Sq3, kLn2), q, 1.0f) * e;
        }
    }
}

template <int D>
__device__ __forceinline__ float sqdist(const float (&ui)[D], const float* __restrict__ uj) {
    float d2 = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float df = ui[k] - uj[k];
        d2 = fmaf(df, df, d2);
    }
    return d2;
}

// ---------------------------------------------------------------- host side

// Prescale factor c_f of a family (see the file comment), in double.
double family_scale(int family);

// Bump allocator over the caller's workspace; with base == nullptr it only
// counts bytes (used by mfgp_workspace_bytes).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Split-j plan for an m x n entry sweep: rows are covered by blocks of
// kRowsPerBlock, columns (j) by `chunks` contiguous ranges of `jchunk`.
constexpr int kBlock = 256;          // threads per block = rows per block
struct SweepPlan {
    int64_t m = 0, n = 0;
    int rowblocks = 0;
    int chunks = 1;
    int64_t jchunk = 0;
};
// Split-j plan of an m x n sweep: 256-row blocks times j-range chunks, about
// `target` blocks per launch.
SweepPlan plan_sweep(int64_t m, int64_t n, int64_t target = 4096);

// Column-block sizes with a compiled register-resident kernel.
int column_block(int t_remaining);

// A product term with Matern or Linear factors (the general product, family
// kFamProd): its prescaled features are the RBF-class ones (periodic circle
// features, then RBF factors) in [0, nr), then each Matern or Linear factor's
// own range [f0[f], f1[f]).  Unit-scale entry:
//   prod_Matern P_nu(q_f) * prod_Linear (u_i . u_j)_f * 2^-(|du|^2_[0,nr) + sum_Matern q_f)
// with q_f = |du| over the factor's features (see prod.hip).
constexpr int kFamProd = 16;
struct ProdDesc {
    int nr = 0;                        // RBF-class features
    int nspec = 0;                     // Matern / Linear factors
    int kind[MFGP_MAX_TERMS] = {};     // MFGP_MATERN12/32/52 or MFGP_LINEAR
    int f0[MFGP_MAX_TERMS] = {};
    int f1[MFGP_MAX_TERMS] = {};
};

// Arguments of the FP32 entry sweep  out = s2 * k(Ur, Uc) V (+ sig2 * Vself).
struct SweepArgs {
    const float* Ur;   // [m, D] prescaled rows
    const float* Uc;   // [n, D] prescaled columns
    const float* V;    // [n, tb] packed column block
    int64_t m, n;
    float* partial;    // [chunks][m][tb] FP32 partial sums
    SweepPlan plan;
    const ProdDesc* pd = nullptr;   // host: the general product's layout (family kFamProd)
};

// Launch the partial-sum sweep for one column block of width tb.
hipError_t launch_sweep_f32(int family, int D, int tb, const SweepArgs& a, hipStream_t s);
// FP64-accumulated sweep (residual recompute): V64 [n, ldv] float64, partial FP64.
struct SweepArgs64 {
    const float* Ur;
    const float* Uc;
    const double* V;
    int ldv;
    int64_t m, n;
    double* partial;   // [chunks][m][tb]
    SweepPlan plan;
    const ProdDesc* pd = nullptr;
};
hipError_t launch_sweep_f64acc(int family, int D, int tb, const SweepArgs64& a, hipStream_t s);

// out[i, c0+c] = s2 * sum_s partial[s][i][c] + sig2 * Vself[i, c0+c]   (Vself may be null)
hipError_t launch_reduce_f32(const float* partial, int chunks, int64_t m, int tb, float s2,
                             float sig2, const float* Vself, int ldv, float* out, int ldo,
                             hipStream_t s);

// Prescale X [n, d] into U [n, D] with per-dimension factors (D == d).
hipError_t launch_prescale(const float* X, int64_t n, int d, const float* fac_host, float* U,
                           hipStream_t s);

}  // namespace mfgp
