// BF16-MFMA form of the entry sweep: the K-tile x V contraction runs on the
// matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation) while the VALU
// generates the kernel entries in FP32 directly in the MFMA A-operand layout.
// This is the precision extension of the fused product: LightGP itself is
// FP32 only (Sec. 5, "Limitations"), and its CG needs only K_y v (Sec. 2).
//
//   x1:  acc += bf(K) bf(V)
//   x2:  acc += bf(K) bf(V) + bf(K) lo(V) + lo(K) bf(V),  lo(a) = bf(a - bf(a))
//
// Operand layout of v_mfma_f32_32x32x16_bf16 (one wave, 64 lanes): lane l
// holds A[l % 32][8 (l / 32) + q] and B[8 (l / 32) + q][l % 32] for q = 0..7,
// and accumulator register r holds C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// Here A = K(rows i, 16 consecutive j), B = V(16 j, 32 columns).
//
// Per wave: RT = 2 row tiles of 32 rows; per block: 4 waves = 256 rows (the
// same block -> (row block, j-chunk) split and partial-sum reduction as the
// FP32 sweeps).  V is converted once per product into "B fragments": for
// j-tile jt and column tile ct, lane l's 8 bf16 values contiguous (16 bytes),
// so a fragment is one 16-byte load per lane.
#include "internal.hpp"
#include "sweep_kernels.hpp"

namespace mfgp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kRT = 2;      // row tiles (of 32 rows) per wave
constexpr int kJT = 16;     // j per MFMA step

bool precision_supported(int p) { return p >= MFGP_FP32 && p <= MFGP_FP32_VALU; }

static inline int col_tiles(int t) { return (t + 31) / 32; }

// Vb[(jt * NT + ct) * 64 + l] = 8 bf16: V[jt*16 + 8(l/32) + q][ct*32 + l%32]
// (hi part, and lo part in Vlo when split); zero outside [n) x [t).
__global__ void pack_vfrag_kernel(const float* __restrict__ V, int64_t n, int t, int nt_tiles,
                                  int64_t njt, int split, bf16x8* __restrict__ Vhi,
                                  bf16x8* __restrict__ Vlo) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = njt * nt_tiles * 64;
    if (idx >= total) return;
    const int l = static_cast<int>(idx % 64);
    const int64_t f = idx / 64;
    const int ct = static_cast<int>(f % nt_tiles);
    const int64_t jt = f / nt_tiles;
    const int c = ct * 32 + (l % 32);
    bf16x8 hi, lo;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t j = jt * kJT + 8 * (l / 32) + q;
        const float v = (j < n && c < t) ? V[j * t + c] : 0.0f;
        const __bf16 h = static_cast<__bf16>(v);
        hi[q] = h;
        lo[q] = static_cast<__bf16>(v - static_cast<float>(h));
    }
    Vhi[idx] = hi;
    if (split) Vlo[idx] = lo;
}

template <int FAM, int D, int NT, int SPLIT>
__global__ __launch_bounds__(kBlock) void sweep_mfma_kernel(
    const float* __restrict__ Ur, const float* __restrict__ Uc, const bf16x8* __restrict__ Vhi,
    const bf16x8* __restrict__ Vlo, int64_t m, int64_t n, int t, int chunks, int64_t jchunk,
    float* __restrict__ partial) {
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int half = lane >> 5;     // which 8 of the 16 j's this lane generates
    const int row_in_tile = lane & 31;
    const int64_t row0 = static_cast<int64_t>(rb) * kBlock + wave * (kRT * 32);

    float ui[kRT][D];
#pragma unroll
    for (int r = 0; r < kRT; ++r) {
        int64_t i = row0 + r * 32 + row_in_tile;
        i = i < m ? i : m - 1;
#pragma unroll
        for (int k = 0; k < D; ++k) ui[r][k] = Ur[i * D + k];
    }
    f32x16 acc[kRT][NT];
#pragma unroll
    for (int r = 0; r < kRT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[r][c][q] = 0.0f;

    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;       // multiple of 16
    int64_t j1 = j0 + jchunk;
    const int64_t npad = (n + kJT - 1) / kJT * kJT;
    j1 = j1 < npad ? j1 : npad;
    for (int64_t jb = j0; jb < j1; jb += kJT) {
        const int64_t jt = jb / kJT;
        bf16x8 bh[NT], bl[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            bh[c] = Vhi[(jt * NT + c) * 64 + lane];
            if (SPLIT) bl[c] = Vlo[(jt * NT + c) * 64 + lane];
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
            bf16x8 ah, al;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float e = kentry<FAM>(sqdist<D>(ui[r], uj[q]));
                const __bf16 h = static_cast<__bf16>(e);
                ah[q] = h;
                if (SPLIT) al[q] = static_cast<__bf16>(e - static_cast<float>(h));
            }
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[c], acc[r][c], 0, 0, 0);
                if (SPLIT) {
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[c], acc[r][c], 0, 0, 0);
                    acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[c], acc[r][c], 0, 0, 0);
                }
            }
        }
    }
    // C layout: register q of lane l -> row 8(q/4) + 4(l/32) + q%4, column l%32.
#pragma unroll
    for (int r = 0; r < kRT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const int col = c * 32 + (lane & 31);
            if (col >= t) continue;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t i = row0 + r * 32 + 8 * (q / 4) + 4 * half + (q % 4);
                if (i < m) partial[(static_cast<int64_t>(ch) * m + i) * t + col] = acc[r][c][q];
            }
        }
}

// ---------------------------------------------------------------- host side

static SweepPlan plan_mfma(int64_t m, int64_t n) {
    SweepPlan p = plan_sweep(m, n);
    // j-ranges in whole 16-wide MFMA steps
    p.jchunk = (p.jchunk + kJT - 1) / kJT * kJT;
    return p;
}

size_t mfma_scratch_bytes(int64_t m, int64_t n, int t, int precision) {
    if (t > 64) t = 64;
    const SweepPlan p = plan_mfma(m, n);
    const int64_t njt = (n + kJT - 1) / kJT;
    const size_t frag = static_cast<size_t>(njt) * col_tiles(t) * 64 * sizeof(bf16x8);
    const size_t part = static_cast<size_t>(p.chunks) * m * t * sizeof(float);
    (void)precision;
    return 2 * frag + part + 4096;
}

template <int FAM, int D>
static hipError_t mfma_fd(int nt, int split, const float* Ur, const float* Uc, const bf16x8* Vhi,
                          const bf16x8* Vlo, int64_t m, int64_t n, int t, const SweepPlan& p,
                          float* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
#define MFGP_MF(NTV, SPV)                                                                          \
    if (nt == NTV && split == SPV) {                                                               \
        hipLaunchKernelGGL((sweep_mfma_kernel<FAM, D, NTV, SPV>), grid, dim3(kBlock), 0, s, Ur, Uc, \
                           Vhi, Vlo, m, n, t, p.chunks, p.jchunk, partial);                        \
        return hipGetLastError();                                                                  \
    }
    MFGP_MF(1, 0) MFGP_MF(1, 1) MFGP_MF(2, 0) MFGP_MF(2, 1)
#undef MFGP_MF
    return hipErrorInvalidValue;
}

template <int FAM>
static hipError_t mfma_f(int D, int nt, int split, const float* Ur, const float* Uc,
                         const bf16x8* Vhi, const bf16x8* Vlo, int64_t m, int64_t n, int t,
                         const SweepPlan& p, float* partial, hipStream_t s) {
    switch (D) {
        case 1: return mfma_fd<FAM, 1>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        case 2: return mfma_fd<FAM, 2>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        case 3: return mfma_fd<FAM, 3>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        case 4: return mfma_fd<FAM, 4>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        case 5: return mfma_fd<FAM, 5>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        case 6: return mfma_fd<FAM, 6>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        case 7: return mfma_fd<FAM, 7>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        case 8: return mfma_fd<FAM, 8>(nt, split, Ur, Uc, Vhi, Vlo, m, n, t, p, partial, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t reduce_partials(const float* partial, int chunks, int64_t m, int t, float s2,
                           float sig2, const float* Vself, float* out, hipStream_t s);

hipError_t apply_mfma(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                      float* out, bool with_noise, const float* Vself, int precision,
                      void* scratch, hipStream_t s) {
    if (t > 64) return hipErrorNotSupported;
    const int nt = col_tiles(t);
    const int split = precision == MFGP_BF16X2 ? 1 : 0;
    const int64_t n = op.n;
    const int64_t njt = (n + kJT - 1) / kJT;
    const SweepPlan p = plan_mfma(m, n);
    char* base = static_cast<char*>(scratch);
    const size_t frag = static_cast<size_t>(njt) * nt * 64 * sizeof(bf16x8);
    bf16x8* Vhi = reinterpret_cast<bf16x8*>(base);
    bf16x8* Vlo = reinterpret_cast<bf16x8*>(base + frag);
    float* partial = reinterpret_cast<float*>(base + 2 * frag);
    const int64_t total = njt * nt * 64;
    hipLaunchKernelGGL(pack_vfrag_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                       0, s, V, n, t, nt, njt, split, Vhi, Vlo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* tok = timing_begin(s);
    switch (op.family) {
        case MFGP_RBF: e = mfma_f<MFGP_RBF>(op.d, nt, split, Ur, op.U, Vhi, Vlo, m, n, t, p, partial, s); break;
        case MFGP_MATERN12: e = mfma_f<MFGP_MATERN12>(op.d, nt, split, Ur, op.U, Vhi, Vlo, m, n, t, p, partial, s); break;
        case MFGP_MATERN32: e = mfma_f<MFGP_MATERN32>(op.d, nt, split, Ur, op.U, Vhi, Vlo, m, n, t, p, partial, s); break;
        default: e = mfma_f<MFGP_MATERN52>(op.d, nt, split, Ur, op.U, Vhi, Vlo, m, n, t, p, partial, s); break;
    }
    {
        const double ent = static_cast<double>(m) * static_cast<double>(n);
        timing_end(tok, s, kSweepMfma, ent, ent * sweep_flops_per_entry(op.family, op.d, t, false));
    }
    if (e != hipSuccess) return e;
    return reduce_partials(partial, p.chunks, m, t, op.s2, with_noise ? op.sig2 : 0.0f,
                           with_noise ? Vself : nullptr, out, s);
}

}  // namespace mfgp
