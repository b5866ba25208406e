// Device body of the BF16-MFMA entry sweep (operand layouts and split forms
// are described in mfma.hip), shared with the batched persistent kernels.
#pragma once

#include "sweep_kernels.hpp"

namespace mfgp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kRT = 2;      // row tiles (of 32 rows) per wave
constexpr int kJT = 16;     // j per MFMA step

// Column 0 on the VALU when the rest fills whole 32-column tiles.
__host__ __device__ inline int vec_cols(int t) { return (t > 1 && t % 32 == 1) ? 1 : 0; }
__host__ __device__ inline int col_tiles(int t) { return (t - vec_cols(t) + 31) / 32; }
__host__ __device__ inline int split_of(int precision) {
    return precision == MFGP_BF16X3 ? 2 : (precision == MFGP_BF16X2 ? 1 : 0);
}

// Exact three-way bf16 split of a binary32 value: v = h + m + l.
__device__ __forceinline__ void split3(float v, __bf16& h, __bf16& m, __bf16& l) {
    h = static_cast<__bf16>(v);
    const float r = v - static_cast<float>(h);
    m = static_cast<__bf16>(r);
    l = static_cast<__bf16>(r - static_cast<float>(m));
}

// One lane's B fragment of j-tile jt, column tile ct of a [n, t] block V:
// 8 bf16 values V[jt*16 + 8(l/32) + q][tv + ct*32 + l%32], zero outside.
__device__ __forceinline__ void vfrag(const float* __restrict__ V, int64_t n, int t, int tv, int64_t jt,
                                      int ct, int l, bf16x8& h8, bf16x8& m8, bf16x8& l8) {
    const int c = tv + ct * 32 + (l % 32);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t j = jt * kJT + 8 * (l / 32) + q;
        const float v = (j < n && c < t) ? V[j * t + c] : 0.0f;
        __bf16 h, mm, ll;
        split3(v, h, mm, ll);
        h8[q] = h;
        m8[q] = mm;
        l8[q] = ll;
    }
}

// One block's share of the BF16 sweep: rows [row_base, row_base + 256) of an
// m x n product over j in [j0, j1) (j0 a multiple of 16); the partial sums of
// row i go to out[(i - row_base) * t + c].
template <int FAM, int D, int NT, int SPLIT, int TV>
__device__ __forceinline__ void mfma_block(const float* __restrict__ Ur, const float* __restrict__ Uc,
                                           const bf16x8* __restrict__ Vh, const bf16x8* __restrict__ Vm,
                                           const bf16x8* __restrict__ Vl, const float* __restrict__ Vy,
                                           int64_t m, int64_t n, int t, int64_t row_base, int64_t j0,
                                           int64_t j1, float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;     // which 8 of the 16 j's this lane generates
    const int row_in_tile = lane & 31;
    const int64_t row0 = row_base + wave * (kRT * 32);

    float ui[kRT][D];
#pragma unroll
    for (int r = 0; r < kRT; ++r) {
        int64_t i = row0 + r * 32 + row_in_tile;
        i = i < m ? i : m - 1;
#pragma unroll
        for (int k = 0; k < D; ++k) ui[r][k] = Ur[i * D + k];
    }
    f32x16 acc[kRT][NT];
    float sv[kRT];
#pragma unroll
    for (int r = 0; r < kRT; ++r) {
        sv[r] = 0.0f;
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[r][c][q] = 0.0f;
    }

    const int64_t npad = (n + kJT - 1) / kJT * kJT;
    j1 = j1 < npad ? j1 : npad;
    for (int64_t jb = j0; jb < j1; jb += kJT) {
        const int64_t jt = jb / kJT;
        bf16x8 bh[NT], bm[NT], bl[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            bh[c] = Vh[(jt * NT + c) * 64 + lane];
            if (SPLIT >= 1) bm[c] = Vm[(jt * NT + c) * 64 + lane];
            if (SPLIT >= 2) bl[c] = Vl[(jt * NT + c) * 64 + lane];
        }
        float y8[8];
        if (TV) {
#pragma unroll
            for (int q = 0; q < 8; ++q) y8[q] = Vy[jb + 8 * half + q];
        }
        // u_j of this lane's 8 j's (clamped: padded j carry V = 0)
        float uj[8][D];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int64_t j = jb + 8 * half + q;
            j = j < n ? j : n - 1;
#pragma unroll
            for (int k = 0; k < D; ++k) uj[q][k] = Uc[j * D + k];
        }
#pragma unroll
        for (int r = 0; r < kRT; ++r) {
            bf16x8 ah, am, al;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float e = kentry<FAM>(sqdist<D>(ui[r], uj[q]));
                if (TV) sv[r] = fmaf(e, y8[q], sv[r]);
                const __bf16 h = static_cast<__bf16>(e);
                ah[q] = h;
                if (SPLIT >= 1) {
                    const float rm = e - static_cast<float>(h);
                    const __bf16 mm = static_cast<__bf16>(rm);
                    am[q] = mm;
                    if (SPLIT >= 2) al[q] = static_cast<__bf16>(rm - static_cast<float>(mm));
                }
            }
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                // smallest terms first
                if (SPLIT >= 2) {
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm[c], acc[r][c], 0, 0, 0);
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[c], acc[r][c], 0, 0, 0);
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[c], acc[r][c], 0, 0, 0);
                }
                if (SPLIT >= 1) {
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm[c], acc[r][c], 0, 0, 0);
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh[c], acc[r][c], 0, 0, 0);
                }
                acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[c], acc[r][c], 0, 0, 0);
            }
        }
    }
    // C layout: register q of lane l -> row 8(q/4) + 4(l/32) + q%4, column l%32.
#pragma unroll
    for (int r = 0; r < kRT; ++r) {
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int col = TV + c * 32 + (lane & 31);
            if (col >= t) continue;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t i = row0 + r * 32 + 8 * (q / 4) + 4 * half + (q % 4);
                if (i < m) out[(i - row_base) * t + col] = acc[r][c][q];
            }
        }
        if (TV) {
            // VALU column: the two lane halves hold the two 8-j halves of row l % 32
            const float v = sv[r] + __shfl_xor(sv[r], 32, 64);
            const int64_t i = row0 + r * 32 + row_in_tile;
            if (half == 0 && i < m) out[(i - row_base) * t] = v;
        }
    }
}


}  // namespace mfgp
