// Device body of the FP32 RBF sweep with the squared distances on FP32 MFMA
// (the Gram form; see gram.hip for the operand layout and the accuracy guard).
#pragma once

#include "hybrid_kernels.hpp"

namespace mfgp {

constexpr int kGJ = 16;   // j per Gram block (one 16 x 16 distance tile per row tile)

// Rows [row_base, row_base + 256) of the n x n RBF product over j in [j0, j1)
// (j0 a multiple of 16).  G [n][DG] holds -2 g_j (g = u - mean(u), zero-padded
// to DG = 4 or 8 dimensions), nrm [n] holds |g_j|^2 and F the V fragments of
// the hybrid sweep with |g_j|^2 as one more value behind the NT + TV
// right-hand-side values of each lane and step (stride WS = NT + TV + 1).
//
// Per 16-j block and row tile of 16 rows one v_mfma_f32_16x16x4_f32 (two for
// DG = 8) produces the 16 x 16 products
//   -2 g_i . g_j = sum_k (-2 g_j[k]) g_i[k]
// from a zero accumulator; the lane takes 2^(2 g_i . g_j) with one exp2, the
// fragment values already carry 2^(-|g_j|^2), and the row's sums are scaled
// by 2^(-|g_i|^2) when they are written (see gram.hip).  Its A operand (16 j x 4 dims)
// takes the block's j in the order pi(row) = 4 (row % 4) + row / 4, so that
// accumulator register s of lane l holds the entry of row i = l % 16 and
// j = j0 + 4 s + l / 16 -- exactly the A operand of contraction step s of the
// hybrid sweep (lane l: row l % 16, j = 4 q + l / 16).  The entries then go
// through the contraction MFMAs (and the TV VALU columns) unchanged.
template <int DG, int NT, int TV>
__device__ __forceinline__ void gram_block(const float* __restrict__ G, const float* __restrict__ nrm,
                                           const float* __restrict__ F, int64_t n, int t, int64_t row_base,
                                           int64_t j0, int64_t j1, float* __restrict__ out) {
    constexpr int W = NT + TV;
    constexpr int WS = W + 1;
    constexpr int H = DG / 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane >> 4;
    const int r16 = lane & 15;
    const int64_t row0 = row_base + wave * (kHRT * 16);

    // B operand of the distance MFMA: lane l holds g_i[4 h + l / 16], i = row l % 16.
    float bi[kHRT][H], ni[kHRT];
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
        int64_t i = row0 + r * 16 + r16;
        i = i < n ? i : n - 1;
#pragma unroll
        for (int h = 0; h < H; ++h) bi[r][h] = -0.5f * G[i * DG + 4 * h + grp];
        ni[r] = nrm[i];
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

    const int64_t npad = (n + kGJ - 1) / kGJ * kGJ;
    j1 = j1 < npad ? j1 : npad;
    const int64_t nblk = j0 < j1 ? (j1 - j0) / kGJ : 0;
    // this lane's j of the A operand within a block (the pi order above)
    const int ja = 4 * (r16 & 3) + (r16 >> 2);

    // Operands of block b: the A operand of the distance MFMA(s) and the four
    // steps' fragments (values behind j >= n are zero; G, nrm and the packed
    // norms repeat row n - 1 there, so every entry stays finite).
    auto load_block = [&](int64_t b, float (&a)[H], float (&f)[4][W]) {
        const int64_t jb = j0 + b * kGJ;
        const float* Gj = G + (jb + ja) * DG + grp;   // rows past n repeat row n - 1
#pragma unroll
        for (int h = 0; h < H; ++h) a[h] = Gj[4 * h];
        const float* Fb = F + (jb / kHK) * (64 * WS);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int w = 0; w < W; ++w) f[s][w] = Fb[(s * 64 + lane) * WS + w];
    };
    const f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
    auto compute_block = [&](const float (&a)[H], const float (&f)[4][W]) {
#pragma unroll
        for (int r = 0; r < kHRT; ++r) {
            f32x4 d2 = zero4;
#pragma unroll
            for (int h = 0; h < H; ++h) d2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[h], bi[r][h], d2, 0, 0, 0);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float e = kentry<MFGP_RBF>(d2[s]);
#pragma unroll
                for (int c = 0; c < NT; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(e, f[s][c], acc[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < TV; ++c) sv[r][c] = fmaf(e, f[s][NT + c], sv[r][c]);
            }
        }
    };
    auto flush = [&]() {
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

    // Ping-pong over two operand sets, one block ahead.  The scheduling
    // barriers keep each prefetch ahead of the other set's compute: without
    // them the compiler sank the loads to their first use, so every block
    // waited out the L2 latency (6.58 -> 6.50 ms here, 7.68 -> 7.28 ms in the
    // direct-difference body, rbf100k t = 33).
    float aa[H], ab[H], fa[4][W], fb[4][W];
    if (nblk > 0) load_block(0, aa, fa);
    int64_t b = 0;
    for (; b + 1 < nblk; b += 2) {
        load_block(b + 1, ab, fb);
        __builtin_amdgcn_sched_barrier(0);
        compute_block(aa, fa);
        __builtin_amdgcn_sched_barrier(0);
        load_block(b + 2 < nblk ? b + 2 : nblk - 1, aa, fa);
        __builtin_amdgcn_sched_barrier(0);
        compute_block(ab, fb);
        __builtin_amdgcn_sched_barrier(0);
        if (((b + 2) & (kSeg / kGJ - 1)) == 0) flush();
    }
    if (b < nblk) compute_block(aa, fa);

    // row factors 2^(-|g_i|^2): of the rows 4 grp + qq of the contraction
    // tiles, and of the lane's own row for the VALU columns
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            int64_t i = row0 + r * 16 + 4 * grp + qq;
            const float ai = __builtin_amdgcn_exp2f(-nrm[i < n ? i : n - 1]);
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const float v = (tot[r][c][qq] + acc[r][c][qq]) * ai;
                if (i < n) out[(i - row_base) * t + TV + 16 * c + r16] = v;
            }
        }
#pragma unroll
        for (int c = 0; c < TV; ++c) {
            float v = tv_tot[r][c] + sv[r][c];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            const int64_t i = row0 + r * 16 + r16;
            v *= __builtin_amdgcn_exp2f(-ni[r]);
            if (grp == 0 && i < n) out[(i - row_base) * t + c] = v;
        }
    }
}

// Two RBF-class terms fused into one sweep (a kernel sum s2_a k_a + s2_b k_b
// whose terms each are RBF on their own features): per 16-j block and row
// tile, one distance MFMA chain per term (Ga / Gb with their norms, as in
// gram_block), the entry e = 2^(-r2_a) + rb 2^(-r2_b) with rb = s2_b / s2_a,
// and one contraction of e for both terms.  F carries |g_j|^2 of both terms
// behind the values (stride WS = NT + TV + 2).  When a term's norms exceed
// the Gram form's bound (gram = false) the squared distances come from
// direct differences of the prescaled points Ua [n][da], Ub [n][db] instead,
// for the same (i, j) of each lane, read from memory as needed.  GRAM
// selects the form for the whole launch (one branch per kernel).
template <int DGA, int DGB, int NT, int TV, bool GRAM>
__device__ __forceinline__ void gram2_block(const float* __restrict__ Ga, const float* __restrict__ nrmA,
                                            const float* __restrict__ Gb, const float* __restrict__ nrmB,
                                            const float* __restrict__ Ua, int da, const float* __restrict__ Ub,
                                            int db, float rb, const float* __restrict__ F, int64_t n,
                                            int t, int64_t row_base, int64_t j0, int64_t j1,
                                            float* __restrict__ out) {
    constexpr int W = NT + TV;
    constexpr int WS = W + 2;
    constexpr int HA = DGA / 4;
    constexpr int HB = DGB / 4;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane >> 4;
    const int r16 = lane & 15;
    const int64_t row0 = row_base + wave * (kHRT * 16);

    float ba[kHRT][HA], bb[kHRT][HB], nia[kHRT], nib[kHRT];
    int64_t irow[kHRT];
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
        int64_t i = row0 + r * 16 + r16;
        i = i < n ? i : n - 1;
        irow[r] = i;
#pragma unroll
        for (int h = 0; h < HA; ++h) ba[r][h] = -0.5f * Ga[i * DGA + 4 * h + grp];
#pragma unroll
        for (int h = 0; h < HB; ++h) bb[r][h] = -0.5f * Gb[i * DGB + 4 * h + grp];
        nia[r] = nrmA[i];
        nib[r] = nrmB[i];
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

    const int64_t npad = (n + kGJ - 1) / kGJ * kGJ;
    j1 = j1 < npad ? j1 : npad;
    const int64_t nblk = j0 < j1 ? (j1 - j0) / kGJ : 0;
    const int ja = 4 * (r16 & 3) + (r16 >> 2);

    auto load_block = [&](int64_t b, float (&aa)[HA], float (&ab)[HB], float (&f)[4][WS]) {
        const int64_t jb = j0 + b * kGJ;
        const float* Gja = Ga + (jb + ja) * DGA + grp;   // rows past n repeat row n - 1
        const float* Gjb = Gb + (jb + ja) * DGB + grp;
#pragma unroll
        for (int h = 0; h < HA; ++h) aa[h] = Gja[4 * h];
#pragma unroll
        for (int h = 0; h < HB; ++h) ab[h] = Gjb[4 * h];
        const float* Fb = F + (jb / kHK) * (64 * WS);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int w = 0; w < WS; ++w) f[s][w] = Fb[(s * 64 + lane) * WS + w];
    };
    auto compute_block = [&](int64_t b, const float (&aa)[HA], const float (&ab)[HB], const float (&f)[4][WS]) {
#pragma unroll
        for (int r = 0; r < kHRT; ++r) {
            f32x4 d2a, d2b;
            if constexpr (GRAM) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    d2a[s] = nia[r] + f[s][W];
                    d2b[s] = nib[r] + f[s][W + 1];
                }
#pragma unroll
                for (int h = 0; h < HA; ++h)
                    d2a = __builtin_amdgcn_mfma_f32_16x16x4f32(aa[h], ba[r][h], d2a, 0, 0, 0);
#pragma unroll
                for (int h = 0; h < HB; ++h)
                    d2b = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[h], bb[r][h], d2b, 0, 0, 0);
            } else {
                const int64_t jb = j0 + b * kGJ;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    int64_t j = jb + 4 * s + grp;
                    j = j < n ? j : n - 1;
                    float sa = 0.0f, sb = 0.0f;
                    for (int k = 0; k < da; ++k) {
                        const float dd = Ua[irow[r] * da + k] - Ua[j * da + k];
                        sa = fmaf(dd, dd, sa);
                    }
                    for (int k = 0; k < db; ++k) {
                        const float dd = Ub[irow[r] * db + k] - Ub[j * db + k];
                        sb = fmaf(dd, dd, sb);
                    }
                    d2a[s] = sa;
                    d2b[s] = sb;
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float e = fmaf(rb, kentry<MFGP_RBF>(d2b[s]), kentry<MFGP_RBF>(d2a[s]));
#pragma unroll
                for (int c = 0; c < NT; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(e, f[s][c], acc[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < TV; ++c) sv[r][c] = fmaf(e, f[s][NT + c], sv[r][c]);
            }
        }
    };
    auto flush = [&]() {
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

    float aa0[HA], ab0[HB], aa1[HA], ab1[HB], fa[4][WS], fb[4][WS];
    if (nblk > 0) load_block(0, aa0, ab0, fa);
    int64_t b = 0;
    for (; b + 1 < nblk; b += 2) {
        load_block(b + 1, aa1, ab1, fb);
        __builtin_amdgcn_sched_barrier(0);
        compute_block(b, aa0, ab0, fa);
        __builtin_amdgcn_sched_barrier(0);
        load_block(b + 2 < nblk ? b + 2 : nblk - 1, aa0, ab0, fa);
        __builtin_amdgcn_sched_barrier(0);
        compute_block(b + 1, aa1, ab1, fb);
        __builtin_amdgcn_sched_barrier(0);
        if (((b + 2) & (kSeg / kGJ - 1)) == 0) flush();
    }
    if (b < nblk) compute_block(b, aa0, ab0, fa);

#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int64_t i = row0 + r * 16 + 4 * grp + qq;
                const float v = tot[r][c][qq] + acc[r][c][qq];
                if (i < n) out[(i - row_base) * t + TV + 16 * c + r16] = v;
            }
#pragma unroll
        for (int c = 0; c < TV; ++c) {
            float v = tv_tot[r][c] + sv[r][c];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            const int64_t i = row0 + r * 16 + r16;
            if (grp == 0 && i < n) out[(i - row_base) * t + c] = v;
        }
    }
}

}  // namespace mfgp
