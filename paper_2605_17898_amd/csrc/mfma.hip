// BF16-MFMA form of the entry sweep: the K-tile x V contraction runs on the
// matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation) while the VALU
// generates the kernel entries in FP32 directly in the MFMA A-operand layout.
// This is the precision extension of the fused product: LightGP itself is
// FP32 only (Sec. 5, "Limitations"), and its CG needs only K_y v (Sec. 2).
//
//   x1:  acc += bf(K) bf(V)
//   x2:  acc += bf(K) bf(V) + bf(K) lo(V) + lo(K) bf(V),  lo(a) = bf(a - bf(a))
//   x3:  a = h + m + l exactly (h = bf(a), m = bf(a - h), l = bf(a - h - m));
//        acc += hh + hm + mh + hl + lh + mm over the pieces of K and V, which
//        drops only terms below 2^-23 |K V|: binary32-class products.
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
// so a fragment is one 16-byte load per lane.  When t = 32 k + 1 (the
// [y, probes] blocks with 32 k probes) column 0 stays on the VALU in FP32
// (one FMA per entry) and the probes fill k whole column tiles.
#include <algorithm>

#include "internal.hpp"
#include "mfma_kernels.hpp"

namespace mfgp {

bool precision_supported(int p) { return p >= MFGP_FP32 && p <= MFGP_FP32_GRAM; }

// Vh[(jt * NT + ct) * 64 + l] = 8 bf16: V[jt*16 + tile_j(l/32, q, perm)][tv + ct*32 + l%32]
// (the first piece; Vm and Vl the second and third when split); zero outside
// [n) x [t).  With tv = 1, Vy[j] = V[j][0] in FP32 (zero for j >= n).  For the
// Gram form (nrm, gmax non-NULL) every value carries the column factor
// 2^(-|g_j|^2) while the launch takes the Gram branch (max |g|^2 <=
// kGramMaxNorm, the sweep's own test) and none otherwise.
__global__ void pack_vfrag_kernel(const float* __restrict__ V, int64_t n, int t, int tv, int nt_tiles,
                                  int64_t njt, int split, int perm, const float* __restrict__ nrm,
                                  const unsigned* __restrict__ gmax, bf16x8* __restrict__ Vh,
                                  bf16x8* __restrict__ Vm, bf16x8* __restrict__ Vl,
                                  float* __restrict__ Vy) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = njt * nt_tiles * 64;
    const float* colnrm = (nrm && __uint_as_float(*gmax) <= kGramMaxNorm) ? nrm : nullptr;
    if (tv && idx < njt * kJT) {
        float y = idx < n ? V[idx * t] : 0.0f;
        if (colnrm) y *= __builtin_amdgcn_exp2f(-colnrm[idx < n ? idx : n - 1]);
        Vy[idx] = y;
    }
    if (idx >= total) return;
    const int l = static_cast<int>(idx % 64);
    const int64_t f = idx / 64;
    const int ct = static_cast<int>(f % nt_tiles);
    const int64_t jt = f / nt_tiles;
    bf16x8 h8, m8, l8;
    vfrag(V, n, t, tv, jt, ct, l, h8, m8, l8, perm != 0, colnrm);
    Vh[idx] = h8;
    if (split >= 1) Vm[idx] = m8;
    if (split >= 2) Vl[idx] = l8;
}

template <int FAM, int D, int NT, int SPLIT, int TV>
__global__ __launch_bounds__(kBlock) void sweep_mfma_kernel(
    const float* __restrict__ Ur, const float* __restrict__ Uc, const bf16x8* __restrict__ Vh,
    const bf16x8* __restrict__ Vm, const bf16x8* __restrict__ Vl, const float* __restrict__ Vy,
    int64_t m, int64_t n, int t, int chunks, int64_t jchunk, float* __restrict__ partial) {
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;       // multiple of 16
    const int64_t row_base = static_cast<int64_t>(rb) * kBlock;
    mfma_block<FAM, D, NT, SPLIT, TV>(Ur, Uc, Vh, Vm, Vl, Vy, m, n, t, row_base, j0, j0 + jchunk,
                                      partial + static_cast<int64_t>(ch) * m * t + row_base * t);
}

// The Gram form for square RBF products (distances on v_mfma_f32_32x32x2_f32,
// see gram_mfma_block): the launch reads the largest centred norm and runs
// the direct-difference body on the same (permuted) fragments above the
// form's accuracy bound.
template <int D, int NT, int SPLIT, int TV>
__global__ __launch_bounds__(kBlock) void sweep_gmfma_kernel(
    const float* __restrict__ U, const float* __restrict__ G, const float* __restrict__ nrm,
    const unsigned* __restrict__ gmax, const bf16x8* __restrict__ Vh, const bf16x8* __restrict__ Vm,
    const bf16x8* __restrict__ Vl, const float* __restrict__ Vy, int64_t n, int t, int chunks, int64_t jchunk,
    float* __restrict__ partial) {
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;       // multiple of 32
    const int64_t row_base = static_cast<int64_t>(rb) * kBlock;
    float* out = partial + static_cast<int64_t>(ch) * n * t + row_base * t;
    if (__uint_as_float(*gmax) <= kGramMaxNorm)
        gram_mfma_block<D <= 4 ? 4 : 8, NT, SPLIT, TV>(G, nrm, Vh, Vm, Vl, Vy, n, t, row_base, j0, j0 + jchunk, out);
    else
        mfma_block<MFGP_RBF, D, NT, SPLIT, TV, true>(U, U, Vh, Vm, Vl, Vy, n, n, t, row_base, j0, j0 + jchunk, out);
}

// ---------------------------------------------------------------- host side

static SweepPlan plan_mfma(int64_t m, int64_t n) {
    SweepPlan p = plan_sweep(m, n);
    // j-ranges in whole 32-j distance tiles (two 16-wide MFMA steps)
    p.jchunk = (p.jchunk + kGB - 1) / kGB * kGB;
    return p;
}

// 16-j tiles covering n rounded up to 32 (the Gram form's distance tiles)
static int64_t mfma_njt(int64_t n) { return (n + kGB - 1) / kGB * (kGB / kJT); }

// Scratch: three fragment arrays (one per split piece), the FP32 column-0
// copy, and the split-j partial sums.
static void mfma_layout(int64_t m, int64_t n, int t, size_t& frag, size_t& ybytes, size_t& part) {
    const SweepPlan p = plan_mfma(m, n);
    const int64_t njt = mfma_njt(n);
    frag = (static_cast<size_t>(njt) * col_tiles(t) * 64 * sizeof(bf16x8) + 255) / 256 * 256;
    ybytes = (static_cast<size_t>(njt) * kJT * sizeof(float) + 255) / 256 * 256;
    part = static_cast<size_t>(p.chunks) * m * t * sizeof(float);
}

size_t mfma_scratch_bytes(int64_t m, int64_t n, int t, int precision) {
    if (t > 65) t = 65;
    size_t frag, ybytes, part;
    mfma_layout(m, n, t, frag, ybytes, part);
    (void)precision;
    return 3 * frag + ybytes + ((part + 255) / 256 * 256) + gram_prep_bytes(n) + 4096;
}

template <int FAM, int D>
static hipError_t mfma_fd(int nt, int split, int tv, const float* Ur, const float* Uc, const bf16x8* Vh,
                          const bf16x8* Vm, const bf16x8* Vl, const float* Vy, int64_t m, int64_t n, int t,
                          const SweepPlan& p, float* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
#define MFGP_MF(NTV, SPV, TVV)                                                                          \
    if (nt == NTV && split == SPV && tv == TVV) {                                                       \
        hipLaunchKernelGGL((sweep_mfma_kernel<FAM, D, NTV, SPV, TVV>), grid, dim3(kBlock), 0, s, Ur, Uc, \
                           Vh, Vm, Vl, Vy, m, n, t, p.chunks, p.jchunk, partial);                       \
        return hipGetLastError();                                                                       \
    }
    MFGP_MF(1, 0, 0) MFGP_MF(1, 1, 0) MFGP_MF(1, 2, 0) MFGP_MF(2, 0, 0) MFGP_MF(2, 1, 0) MFGP_MF(2, 2, 0)
    MFGP_MF(1, 0, 1) MFGP_MF(1, 1, 1) MFGP_MF(1, 2, 1) MFGP_MF(2, 0, 1) MFGP_MF(2, 1, 1) MFGP_MF(2, 2, 1)
#undef MFGP_MF
    return hipErrorInvalidValue;
}

template <int D>
static hipError_t gmfma_d(int nt, int split, int tv, const float* U, const GramPrep& g, const bf16x8* Vh,
                          const bf16x8* Vm, const bf16x8* Vl, const float* Vy, int64_t n, int t, const SweepPlan& p,
                          float* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
#define MFGP_GMF(NTV, SPV, TVV)                                                                        \
    if (nt == NTV && split == SPV && tv == TVV) {                                                      \
        hipLaunchKernelGGL((sweep_gmfma_kernel<D, NTV, SPV, TVV>), grid, dim3(kBlock), 0, s, U, g.G, g.nrm, \
                           g.gmax, Vh, Vm, Vl, Vy, n, t, p.chunks, p.jchunk, partial);                 \
        return hipGetLastError();                                                                      \
    }
    MFGP_GMF(1, 0, 0) MFGP_GMF(1, 1, 0) MFGP_GMF(1, 2, 0) MFGP_GMF(2, 0, 0) MFGP_GMF(2, 1, 0) MFGP_GMF(2, 2, 0)
    MFGP_GMF(1, 0, 1) MFGP_GMF(1, 1, 1) MFGP_GMF(1, 2, 1) MFGP_GMF(2, 0, 1) MFGP_GMF(2, 1, 1) MFGP_GMF(2, 2, 1)
#undef MFGP_GMF
    return hipErrorInvalidValue;
}

template <int FAM>
static hipError_t mfma_f(int D, int nt, int split, int tv, const float* Ur, const float* Uc,
                         const bf16x8* Vh, const bf16x8* Vm, const bf16x8* Vl, const float* Vy, int64_t m,
                         int64_t n, int t, const SweepPlan& p, float* partial, hipStream_t s) {
    switch (D) {
#define MFGP_MD(DV) \
        case DV: return mfma_fd<FAM, DV>(nt, split, tv, Ur, Uc, Vh, Vm, Vl, Vy, m, n, t, p, partial, s);
        MFGP_MD(1) MFGP_MD(2) MFGP_MD(3) MFGP_MD(4) MFGP_MD(5) MFGP_MD(6) MFGP_MD(7) MFGP_MD(8)
#undef MFGP_MD
        default: return hipErrorInvalidValue;
    }
}

hipError_t reduce_partials(const float* partial, int chunks, int64_t m, int t, float s2,
                           float sig2, const float* Vself, float* out, hipStream_t s);

hipError_t apply_mfma(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                      float* out, bool with_noise, const float* Vself, int precision,
                      void* scratch, hipStream_t s) {
    if (t > 65) return hipErrorNotSupported;
    const int tv = vec_cols(t);
    const int nt = col_tiles(t);
    if (nt < 1 || nt > 2) return hipErrorNotSupported;
    const int split = split_of(precision);
    const int64_t n = op.n;
    const int64_t njt = mfma_njt(n);
    const SweepPlan p = plan_mfma(m, n);
    size_t frag, ybytes, part;
    mfma_layout(m, n, t, frag, ybytes, part);
    char* base = static_cast<char*>(scratch);
    bf16x8* Vh = reinterpret_cast<bf16x8*>(base);
    bf16x8* Vm = reinterpret_cast<bf16x8*>(base + frag);
    bf16x8* Vl = reinterpret_cast<bf16x8*>(base + 2 * frag);
    float* Vy = reinterpret_cast<float*>(base + 3 * frag);
    float* partial = reinterpret_cast<float*>(base + 3 * frag + ybytes);
    void* prep = base + 3 * frag + ybytes + (part + 255) / 256 * 256;
    // Gram-form distances for square RBF products at n >= kGramMinN (as the
    // FP32 form), with the fragments in the distance tiles' j order.
    const bool gram = op.family == MFGP_RBF && Ur == op.U && m == n && n >= kGramMinN && op.d >= 1 && op.d <= 8;
    GramPrep gp;
    if (gram && op.gram_pre) {
        gp = *op.gram_pre;   // prepared once by the solver
    } else if (gram) {
        hipError_t ge = gram_prepare(op, prep, gp, s);
        if (ge != hipSuccess) return ge;
    }
    const int64_t total = std::max<int64_t>(njt * nt * 64, njt * kJT);
    hipLaunchKernelGGL(pack_vfrag_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                       0, s, V, n, t, tv, nt, njt, split, gram ? 1 : 0, gram ? gp.nrm : nullptr,
                       gram ? gp.gmax : nullptr, Vh, Vm, Vl, Vy);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* tok = timing_begin(s);
    if (gram) {
        switch (op.d) {
#define MFGP_GD(DV) \
            case DV: e = gmfma_d<DV>(nt, split, tv, op.U, gp, Vh, Vm, Vl, Vy, n, t, p, partial, s); break;
            MFGP_GD(1) MFGP_GD(2) MFGP_GD(3) MFGP_GD(4) MFGP_GD(5) MFGP_GD(6) MFGP_GD(7) MFGP_GD(8)
#undef MFGP_GD
            default: e = hipErrorInvalidValue;
        }
    } else {
        switch (op.family) {
            case MFGP_RBF:
                e = mfma_f<MFGP_RBF>(op.d, nt, split, tv, Ur, op.U, Vh, Vm, Vl, Vy, m, n, t, p, partial, s);
                break;
            case MFGP_MATERN12:
                e = mfma_f<MFGP_MATERN12>(op.d, nt, split, tv, Ur, op.U, Vh, Vm, Vl, Vy, m, n, t, p, partial, s);
                break;
            case MFGP_MATERN32:
                e = mfma_f<MFGP_MATERN32>(op.d, nt, split, tv, Ur, op.U, Vh, Vm, Vl, Vy, m, n, t, p, partial, s);
                break;
            default:
                e = mfma_f<MFGP_MATERN52>(op.d, nt, split, tv, Ur, op.U, Vh, Vm, Vl, Vy, m, n, t, p, partial, s);
                break;
        }
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
