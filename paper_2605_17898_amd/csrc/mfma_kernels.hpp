// Device body of the BF16-MFMA entry sweep (operand layouts and split forms
// are described in mfma.hip), shared with the batched persistent kernels.
#pragma once

#include "sweep_kernels.hpp"

namespace mfgp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4v;

constexpr int kRT = 2;      // row tiles (of 32 rows) per wave
constexpr int kJT = 16;     // j per MFMA step

// Column 0 on the VALU when the rest fills whole 32-column tiles.
__host__ __device__ inline int vec_cols(int t) { return (t > 1 && t % 32 == 1) ? 1 : 0; }
__host__ __device__ inline int col_tiles(int t) { return (t - vec_cols(t) + 31) / 32; }
__host__ __device__ inline int split_of(int precision) {
    return precision == MFGP_BF16X3 ? 2 : (precision == MFGP_BF16X2 ? 1 : 0);
}

typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// The split pieces of eight binary32 entries, two values per conversion
// (v_cvt_pk_bf16_f32, round to nearest even; the same values as converting
// them one at a time, half the conversions): h = bf(e), and for SPLIT >= 1
// m = bf(e - h), for SPLIT >= 2 l = bf(e - h - m); the differences are exact
// in binary32 (two v_sub_f32, no packed FP32).
template <int SPLIT>
__device__ __forceinline__ void split8(const float (&e)[8], bf16x8& h8, bf16x8& m8, bf16x8& l8) {
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        const f32x2v v = {e[q], e[q + 1]};
        const bf16x2v h = __builtin_convertvector(v, bf16x2v);
        h8[q] = h[0];
        h8[q + 1] = h[1];
        if (SPLIT >= 1) {
            const f32x2v r = v - __builtin_convertvector(h, f32x2v);
            const bf16x2v m = __builtin_convertvector(r, bf16x2v);
            m8[q] = m[0];
            m8[q + 1] = m[1];
            if (SPLIT >= 2) {
                const f32x2v r2 = r - __builtin_convertvector(m, f32x2v);
                const bf16x2v l = __builtin_convertvector(r2, bf16x2v);
                l8[q] = l[0];
                l8[q + 1] = l[1];
            }
        }
    }
}

// Exact three-way bf16 split of a binary32 value: v = h + m + l.
__device__ __forceinline__ void split3(float v, __bf16& h, __bf16& m, __bf16& l) {
    h = static_cast<__bf16>(v);
    const float r = v - static_cast<float>(h);
    m = static_cast<__bf16>(r);
    l = static_cast<__bf16>(r - static_cast<float>(m));
}

// The j of k = 8 h + q (lane half h = l / 32) within a 16-j tile: k itself,
// or, in the order of the Gram-form bf16 sweep, 4 h + (q % 4) + 8 (q / 4) --
// the rows that registers q of a v_mfma_f32_32x32x2_f32 distance tile hold
// (see gram_mfma_block).
__host__ __device__ inline int tile_j(int h, int q, bool perm) {
    return perm ? 4 * h + (q & 3) + 8 * (q >> 2) : 8 * h + q;
}

// One lane's B fragment of j-tile jt, column tile ct of a [n, t] block V:
// 8 bf16 values V[jt*16 + tile_j(l/32, q)][tv + ct*32 + l%32], zero outside.
// With colnrm non-NULL the values carry the Gram form's column factor
// 2^(-colnrm[j]).
__device__ __forceinline__ void vfrag(const float* __restrict__ V, int64_t n, int t, int tv, int64_t jt,
                                      int ct, int l, bf16x8& h8, bf16x8& m8, bf16x8& l8, bool perm = false,
                                      const float* __restrict__ colnrm = nullptr) {
    const int c = tv + ct * 32 + (l % 32);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t j = jt * kJT + tile_j(l / 32, q, perm);
        float v = (j < n && c < t) ? V[j * t + c] : 0.0f;
        if (colnrm) v *= __builtin_amdgcn_exp2f(-colnrm[j < n ? j : n - 1]);
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
template <int FAM, int D, int NT, int SPLIT, int TV, bool PERM = false>
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
            for (int q = 0; q < 8; ++q) y8[q] = Vy[jb + tile_j(half, q, PERM)];
        }
        // u_j of this lane's 8 j's (clamped: padded j carry V = 0)
        float uj[8][D];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int64_t j = jb + tile_j(half, q, PERM);
            j = j < n ? j : n - 1;
#pragma unroll
            for (int k = 0; k < D; ++k) uj[q][k] = Uc[j * D + k];
        }
#pragma unroll
        for (int r = 0; r < kRT; ++r) {
            bf16x8 ah, am, al;
            float e8[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                e8[q] = kentry<FAM>(sqdist<D>(ui[r], uj[q]));
                if (TV) sv[r] = fmaf(e8[q], y8[q], sv[r]);
            }
            split8<SPLIT>(e8, ah, am, al);
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


constexpr int kGB = 32;   // j per distance tile of the Gram-form bf16 sweep

// Rows [row_base, row_base + 256) of the n x n RBF product over j in [j0, j1)
// (j0 a multiple of 32) in the Gram form: per 32 j and row tile of 32 rows,
// DG / 2 v_mfma_f32_32x32x2_f32 give the products
//   -2 g_i . g_j = sum_k (-2 g_j[k]) g_i[k]
// (A = -2 g_j: 32 j x 2 dims, B = g_i: 2 dims x 32 rows, zero accumulator);
// the factored entry 2^(2 g_i . g_j) is split and contracted with fragments
// that carry 2^(-|g_j|^2), and the row's sums take 2^(-|g_i|^2) at the end
// (the factoring of gram.hip).  Register R of lane l then holds the entry of row
// i = l % 32 and j = j0 + 8 (R / 4) + 4 (l / 32) + R % 4: registers 0..7 are
// exactly the A operand of the first 16-j contraction step and 8..15 of the
// second when the B fragments list their j in the tile_j(.., true) order.
// G, nrm and the fragments as in gram_prepare / pack_vfrag_kernel (perm).
template <int DG, int NT, int SPLIT, int TV>
__device__ __forceinline__ void gram_mfma_block(const float* __restrict__ G, const float* __restrict__ nrm,
                                                const bf16x8* __restrict__ Vh, const bf16x8* __restrict__ Vm,
                                                const bf16x8* __restrict__ Vl, const float* __restrict__ Vy,
                                                int64_t n, int t, int64_t row_base, int64_t j0, int64_t j1,
                                                float* __restrict__ out) {
    constexpr int H = DG / 2;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;
    const int r32 = lane & 31;
    const int64_t row0 = row_base + wave * (kRT * 32);

    float bi[kRT][H], ni[kRT];
#pragma unroll
    for (int r = 0; r < kRT; ++r) {
        int64_t i = row0 + r * 32 + r32;
        i = i < n ? i : n - 1;
#pragma unroll
        for (int h = 0; h < H; ++h) bi[r][h] = -0.5f * G[i * DG + 2 * h + half];
        ni[r] = nrm[i];
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

    f32x16 zero16;
#pragma unroll
    for (int q = 0; q < 16; ++q) zero16[q] = 0.0f;
    const int64_t npad = (n + kGB - 1) / kGB * kGB;
    j1 = j1 < npad ? j1 : npad;
    for (int64_t jb = j0; jb < j1; jb += kGB) {
        // G and nrm hold whole tiles (rows past n repeat row n - 1, whose V is
        // zero), so the tile is read without clamping
        float a[H];
        const float* Gb = G + (jb + r32) * DG + half;
#pragma unroll
        for (int h = 0; h < H; ++h) a[h] = Gb[2 * h];
        // y (with its column factor) at this lane's 16 j's: four runs of 4
        // consecutive j
        float yj[16];
        const float* yb = Vy + jb + 4 * half;
        if (TV) {
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) {
                const f32x4v yv = *reinterpret_cast<const f32x4v*>(yb + 8 * g4);
#pragma unroll
                for (int q = 0; q < 4; ++q) yj[4 * g4 + q] = yv[q];
            }
        }
        bf16x8 bh[2][NT], bm[2][NT], bl[2][NT];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const int64_t f = ((jb / kJT + u) * NT + c) * 64 + lane;
                bh[u][c] = Vh[f];
                if (SPLIT >= 1) bm[u][c] = Vm[f];
                if (SPLIT >= 2) bl[u][c] = Vl[f];
            }
#pragma unroll
        for (int r = 0; r < kRT; ++r) {
            f32x16 d2 = zero16;
#pragma unroll
            for (int h = 0; h < H; ++h) d2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[h], bi[r][h], d2, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                bf16x8 ah, am, al;
                float e8[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    e8[q] = kentry<MFGP_RBF>(d2[8 * u + q]);
                    if (TV) sv[r] = fmaf(e8[q], yj[8 * u + q], sv[r]);
                }
                split8<SPLIT>(e8, ah, am, al);
#pragma unroll
                for (int c = 0; c < NT; ++c) {
                    if (SPLIT >= 2) {
                        acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm[u][c], acc[r][c], 0, 0, 0);
                        acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[u][c], acc[r][c], 0, 0, 0);
                        acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[u][c], acc[r][c], 0, 0, 0);
                    }
                    if (SPLIT >= 1) {
                        acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm[u][c], acc[r][c], 0, 0, 0);
                        acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh[u][c], acc[r][c], 0, 0, 0);
                    }
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[u][c], acc[r][c], 0, 0, 0);
                }
            }
        }
    }
    // row factors 2^(-|g_i|^2) of the rows register q holds (and of the
    // lane's own row for the VALU column)
#pragma unroll
    for (int r = 0; r < kRT; ++r) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t i = row0 + r * 32 + 8 * (q / 4) + 4 * half + (q % 4);
            const float ai = __builtin_amdgcn_exp2f(-nrm[i < n ? i : n - 1]);
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const int col = TV + c * 32 + (lane & 31);
                if (col < t && i < n) out[(i - row_base) * t + col] = acc[r][c][q] * ai;
            }
        }
        if (TV) {
            const float v = (sv[r] + __shfl_xor(sv[r], 32, 64)) * __builtin_amdgcn_exp2f(-ni[r]);
            const int64_t i = row0 + r * 32 + r32;
            if (half == 0 && i < n) out[(i - row_base) * t] = v;
        }
    }
}

}  // namespace mfgp
