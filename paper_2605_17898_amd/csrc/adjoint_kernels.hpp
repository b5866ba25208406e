// Adjoint-sweep device functions shared by the single-problem and batched
// gradient kernels (see adjoint.hip for the mathematics).
#pragma once

#include "hybrid_kernels.hpp"

namespace mfgp {

struct ColW {
    float w[MFGP_MAX_T];
};

template <int FAM>
__device__ __forceinline__ void kentry_and_dfac(float d2, float& kv, float& g) {
    if constexpr (FAM == MFGP_RBF) {
        kv = __builtin_amdgcn_exp2f(-d2);
        g = kv;
    } else {
        const float q = __builtin_amdgcn_sqrtf(d2);
        const float e = __builtin_amdgcn_exp2f(-q);
        if constexpr (FAM == MFGP_MATERN12) {
            kv = e;
            g = q > 0.0f ? e * __builtin_amdgcn_rcpf(q) : 0.0f;
        } else if constexpr (FAM == MFGP_MATERN32) {
            kv = fmaf(q, kLn2, 1.0f) * e;
            g = e;
        } else {
            kv = fmaf(fmaf(q, kLn2Sq3, kLn2), q, 1.0f) * e;
            g = fmaf(q, kLn2, 1.0f) * e;
        }
    }
}

// Lane sums over cnt columns j of W_ij g(q) du_k^2 (k < D) and W_ij k^ into
// v[0..D] (FP64 after two-level FP32 accumulation); ai holds w_c A_ic.
template <int FAM, int D, int TB>
__device__ __forceinline__ void adjoint_rows(const float (&ui)[D], const float (&ai)[TB],
                                             const float* __restrict__ uc,
                                             const float* __restrict__ bc, int cnt,
                                             double (&v)[D + 1]) {
    float g[D], gs = 0.0f, tg[D], ts = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        g[k] = 0.0f;
        tg[k] = 0.0f;
    }
    for (int q = 0; q < cnt; ++q) {
        if (q % kSeg == 0 && q > 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                tg[k] += g[k];
                g[k] = 0.0f;
            }
            ts += gs;
            gs = 0.0f;
        }
        const float* uj = uc + q * D;
        float df[D];
        float d2 = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            df[k] = ui[k] - uj[k];
            d2 = fmaf(df[k], df[k], d2);
        }
        float kv, gf;
        kentry_and_dfac<FAM>(d2, kv, gf);
        float wij = 0.0f;
#pragma unroll
        for (int c = 0; c < TB; ++c) wij = fmaf(ai[c], bc[q * TB + c], wij);
        gs = fmaf(wij, kv, gs);
        const float wd = wij * gf;
#pragma unroll
        for (int k = 0; k < D; ++k) g[k] = fmaf(wd * df[k], df[k], g[k]);
    }
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = static_cast<double>(tg[k]) + static_cast<double>(g[k]);
    v[D] = static_cast<double>(ts) + static_cast<double>(gs);
}

// FP64 block reduction of v[0..W-1] (wave butterfly, then the 4 wave sums in
// order); thread k < W writes the block total of component k to out[k].
template <int W>
__device__ __forceinline__ void block_sum_write(double (&v)[W], double* red, double* out) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[k] = x;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) red[wave * W + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < W) {
        double s = 0.0;
        for (int q = 0; q < kBlock / 64; ++q) s += red[q * W + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

}  // namespace mfgp
