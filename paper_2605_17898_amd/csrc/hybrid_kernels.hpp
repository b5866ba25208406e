// Device body of the FP32 sweep with the contraction on FP32 MFMA (see
// hybrid.hip for the operand layout), shared with the batched kernels.
#pragma once

#include "sweep_kernels.hpp"

namespace mfgp {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kHRT = 4;     // row tiles of 16 per wave
constexpr int kHK = 4;      // j per MFMA step

// One block's share of the hybrid sweep: rows [row_base, row_base + 256) of
// an m x n product over j in [j0, j1) (j0 a multiple of 4); the partial sums of
// row i go to out[(i - row_base) * t + c].  Shared by the single-problem and
// the batched (persistent) kernels.  WS is the per-lane stride of a step's
// fragment (NT + TV, or more when a caller packs extra values behind them).
template <int FAM, int D, int NT, int TV, int WS = NT + TV>
__device__ __forceinline__ void hyb_block(const float* __restrict__ Ur, const float* __restrict__ Uc,
                                          const float* __restrict__ F, int64_t m, int64_t n, int t,
                                          int64_t row_base, int64_t j0, int64_t j1,
                                          float* __restrict__ out) {
    constexpr int W = NT + TV;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane >> 4;       // which of the 4 j's of a step this lane generates
    const int r16 = lane & 15;
    const int64_t row0 = row_base + wave * (kHRT * 16);

    float ui[kHRT][D];
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
        int64_t i = row0 + r * 16 + r16;
        i = i < m ? i : m - 1;
#pragma unroll
        for (int k = 0; k < D; ++k) ui[r][k] = Ur[i * D + k];
    }
    f32x4 acc[kHRT][NT > 0 ? NT : 1], tot[kHRT][NT > 0 ? NT : 1];
    float sv[kHRT][TV > 0 ? TV : 1], tv_tot[kHRT][TV > 0 ? TV : 1];
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc[r][c][q] = 0.0f;
                tot[r][c][q] = 0.0f;
            }
#pragma unroll
        for (int c = 0; c < TV; ++c) {
            sv[r][c] = 0.0f;
            tv_tot[r][c] = 0.0f;
        }
    }

    const int64_t npad = (n + kHK - 1) / kHK * kHK;
    j1 = j1 < npad ? j1 : npad;
    const int64_t q0 = j0 / kHK;
    const int64_t nst = j0 < j1 ? (j1 - j0) / kHK : 0;     // MFMA steps of this chunk
    // Steps whose four j are all < n need no clamping; at most the last step
    // of the last chunk is ragged.
    const int64_t qfull = n / kHK;
    int64_t nfull = qfull - q0;
    nfull = nfull < 0 ? 0 : (nfull < nst ? nfull : nst);

    // Operands of one step: this lane's fragment of V and u_j (j = 4 q + grp),
    // addressed as a wave-uniform base plus a fixed per-lane offset.
    auto load_step = [&](int64_t st, float (&f)[W], float (&u)[D]) {
        const int64_t q = q0 + st;
        const float* Fq = F + q * (64 * WS);
#pragma unroll
        for (int w = 0; w < W; ++w) f[w] = Fq[lane * WS + w];
        const float* Uq = Uc + q * (kHK * D);
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = Uq[grp * D + k];
    };
    auto load_step_clamped = [&](int64_t st, float (&f)[W], float (&u)[D]) {
        const int64_t q = q0 + st;
#pragma unroll
        for (int w = 0; w < W; ++w) f[w] = F[(q * 64 + lane) * WS + w];
        int64_t j = q * kHK + grp;
        j = j < n ? j : n - 1;    // padded j carry V = 0
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = Uc[j * D + k];
    };
    auto compute_step = [&](const float (&f)[W], const float (&u)[D]) {
#pragma unroll
        for (int r = 0; r < kHRT; ++r) {
            const float e = kentry<FAM>(sqdist<D>(ui[r], u));
#pragma unroll
            for (int c = 0; c < NT; ++c)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(e, f[c], acc[r][c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < TV; ++c) sv[r][c] = fmaf(e, f[NT + c], sv[r][c]);
        }
    };
    auto flush = [&]() {   // two-level accumulation, as in the VALU sweeps
#pragma unroll
        for (int r = 0; r < kHRT; ++r) {
#pragma unroll
            for (int c = 0; c < NT; ++c)
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    tot[r][c][qq] += acc[r][c][qq];
                    acc[r][c][qq] = 0.0f;
                }
#pragma unroll
            for (int c = 0; c < TV; ++c) {
                tv_tot[r][c] += sv[r][c];
                sv[r][c] = 0.0f;
            }
        }
    };

    // Ping-pong over two operand sets: the loads of one step are in flight
    // while the other step's entries and MFMAs run.  The scheduling barriers
    // keep the prefetch ahead of the compute (the compiler otherwise sank the
    // loads to their first use: 7.68 -> 7.28 ms at rbf100k, t = 33).
    float fa[W], ua[D], fb[W], ub[D];
    if (nfull > 0) load_step(0, fa, ua);
    int64_t st = 0;
    for (; st + 1 < nfull; st += 2) {
        load_step(st + 1, fb, ub);
        __builtin_amdgcn_sched_barrier(0);
        compute_step(fa, ua);
        __builtin_amdgcn_sched_barrier(0);
        load_step(st + 2 < nfull ? st + 2 : nfull - 1, fa, ua);
        __builtin_amdgcn_sched_barrier(0);
        compute_step(fb, ub);
        __builtin_amdgcn_sched_barrier(0);
        if (((st + 2) & (kSeg / kHK - 1)) == 0) flush();
    }
    if (st < nfull) {
        compute_step(fa, ua);
        ++st;
    }
    for (; st < nst; ++st) {     // the ragged tail (at most one step)
        load_step_clamped(st, fa, ua);
        compute_step(fa, ua);
    }
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
        // MFMA columns: register qq of lane l -> row 4 (l/16) + qq, column l % 16
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int64_t i = row0 + r * 16 + 4 * grp + qq;
                const float v = tot[r][c][qq] + acc[r][c][qq];
                if (i < m) out[(i - row_base) * t + TV + 16 * c + r16] = v;
            }
        // VALU columns: sum the 4 lane groups (j offsets) of row r16
#pragma unroll
        for (int c = 0; c < TV; ++c) {
            float v = tv_tot[r][c] + sv[r][c];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            const int64_t i = row0 + r * 16 + r16;
            if (grp == 0 && i < m) out[(i - row_base) * t + c] = v;
        }
    }
}

}  // namespace mfgp
