// FP32 entry sweep with the K-tile x V contraction on the FP32 matrix cores.
//
// For many right-hand sides the contraction (2t FLOP per entry) dominates the
// VALU sweep.  Here the columns split into NT tiles of 16 contracted with
// v_mfma_f32_16x16x4_f32 (FP32 inputs, FP32 accumulation: the same
// arithmetic class as the VALU FMAs) and TV leftover columns (t = 16 NT + TV,
// e.g. the y column of [y, probes]) that stay on the VALU.  The VALU only
// generates entries, directly in the MFMA A-operand layout.
//
// v_mfma_f32_16x16x4_f32 (one wave, 64 lanes): lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator register r holds C[4 (l / 16) + r][l % 16].
// With A = K(16 rows, 4 consecutive j) each lane generates exactly one entry
// per MFMA step: row l % 16 of the tile, column j0 + l / 16.
//
// A wave owns RT = 4 row tiles (64 rows), a block 4 waves (256 rows), with the
// same block -> (row block, j-chunk) split and fixed-order partial reduction
// as the other sweeps.  V is repacked once per product into per-step
// fragments: for step q (4 j's) and lane l, NT values V[4q + l/16][TV + 16 w +
// l%16] followed by the TV leftover values V[4q + l/16][0..TV), so a lane
// fetches all its right-hand-side operands of a step with one load.
#include "hybrid_kernels.hpp"
#include "internal.hpp"

namespace mfgp {

__global__ void pack_hfrag_kernel(const float* __restrict__ V, int64_t n, int t, int nt, int tv,
                                  int64_t nsteps, float* __restrict__ F) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int W = nt + tv;
    if (idx >= nsteps * 64 * W) return;
    const int w = static_cast<int>(idx % W);
    const int64_t lq = idx / W;
    const int l = static_cast<int>(lq % 64);
    const int64_t q = lq / 64;
    const int64_t j = q * kHK + l / 16;
    const int c = w < nt ? tv + 16 * w + (l % 16) : w - nt;
    F[idx] = (j < n) ? V[j * t + c] : 0.0f;
}

template <int FAM, int D, int NT, int TV>
__global__ __launch_bounds__(kBlock) void sweep_hyb_kernel(
    const float* __restrict__ Ur, const float* __restrict__ Uc, const float* __restrict__ F,
    int64_t m, int64_t n, int t, int chunks, int64_t jchunk, float* __restrict__ partial) {
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;          // multiple of kHK
    hyb_block<FAM, D, NT, TV>(Ur, Uc, F, m, n, t, static_cast<int64_t>(rb) * kBlock, j0, j0 + jchunk,
                              partial + static_cast<int64_t>(ch) * m * t + static_cast<int64_t>(rb) * kBlock * t);
}

// (NT, TV) pairs with a compiled kernel: t = 16 NT + TV.
static bool hybrid_shape(int t, int& nt, int& tv) {
    nt = t / 16;
    tv = t % 16;
    return nt >= 1 && nt <= 4 && tv <= 1;
}

bool hybrid_supported(int t) {
    int nt, tv;
    return hybrid_shape(t, nt, tv);
}

static SweepPlan plan_hybrid(int64_t m, int64_t n) {
    SweepPlan p = plan_sweep(m, n);
    p.jchunk = (p.jchunk + kHK - 1) / kHK * kHK;
    return p;
}

size_t hybrid_scratch_bytes(int64_t m, int64_t n, int t) {
    int nt, tv;
    if (!hybrid_shape(t, nt, tv)) return 0;
    const SweepPlan p = plan_hybrid(m, n);
    const int64_t nsteps = (n + kHK - 1) / kHK;
    const size_t frag = static_cast<size_t>(nsteps) * 64 * (nt + tv) * sizeof(float);
    const size_t part = static_cast<size_t>(p.chunks) * m * t * sizeof(float);
    return frag + part + 1024;
}

template <int FAM, int D>
static hipError_t hyb_fd(int nt, int tv, const float* Ur, const float* Uc, const float* F, int64_t m,
                         int64_t n, int t, const SweepPlan& p, float* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
#define MFGP_HYB_CASE(NTV, TVV)                                                                   \
    if (nt == NTV && tv == TVV) {                                                                 \
        hipLaunchKernelGGL((sweep_hyb_kernel<FAM, D, NTV, TVV>), grid, dim3(kBlock), 0, s, Ur, Uc, \
                           F, m, n, t, p.chunks, p.jchunk, partial);                              \
        return hipGetLastError();                                                                 \
    }
    MFGP_HYB_CASE(1, 0) MFGP_HYB_CASE(1, 1) MFGP_HYB_CASE(2, 0) MFGP_HYB_CASE(2, 1)
    MFGP_HYB_CASE(3, 0) MFGP_HYB_CASE(3, 1) MFGP_HYB_CASE(4, 0) MFGP_HYB_CASE(4, 1)
#undef MFGP_HYB_CASE
    return hipErrorInvalidValue;
}

template <int FAM>
static hipError_t hyb_f(int D, int nt, int tv, const float* Ur, const float* Uc, const float* F, int64_t m,
                        int64_t n, int t, const SweepPlan& p, float* partial, hipStream_t s) {
    switch (D) {
        case 1: return hyb_fd<FAM, 1>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        case 2: return hyb_fd<FAM, 2>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        case 3: return hyb_fd<FAM, 3>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        case 4: return hyb_fd<FAM, 4>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        case 5: return hyb_fd<FAM, 5>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        case 6: return hyb_fd<FAM, 6>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        case 7: return hyb_fd<FAM, 7>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        case 8: return hyb_fd<FAM, 8>(nt, tv, Ur, Uc, F, m, n, t, p, partial, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t reduce_partials(const float* partial, int chunks, int64_t m, int t, float s2,
                           float sig2, const float* Vself, float* out, hipStream_t s);

hipError_t apply_hybrid(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                        float* out, bool with_noise, const float* Vself, void* scratch, hipStream_t s) {
    int nt, tv;
    if (!hybrid_shape(t, nt, tv)) return hipErrorNotSupported;
    const int64_t n = op.n;
    const int64_t nsteps = (n + kHK - 1) / kHK;
    const SweepPlan p = plan_hybrid(m, n);
    char* base = static_cast<char*>(scratch);
    float* F = reinterpret_cast<float*>(base);
    const size_t frag = static_cast<size_t>(nsteps) * 64 * (nt + tv) * sizeof(float);
    float* partial = reinterpret_cast<float*>(base + ((frag + 255) / 256) * 256);
    const int64_t total = nsteps * 64 * (nt + tv);
    hipLaunchKernelGGL(pack_hfrag_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0,
                       s, V, n, t, nt, tv, nsteps, F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* tok = timing_begin(s);
    switch (op.family) {
        case MFGP_RBF: e = hyb_f<MFGP_RBF>(op.d, nt, tv, Ur, op.U, F, m, n, t, p, partial, s); break;
        case MFGP_MATERN12: e = hyb_f<MFGP_MATERN12>(op.d, nt, tv, Ur, op.U, F, m, n, t, p, partial, s); break;
        case MFGP_MATERN32: e = hyb_f<MFGP_MATERN32>(op.d, nt, tv, Ur, op.U, F, m, n, t, p, partial, s); break;
        default: e = hyb_f<MFGP_MATERN52>(op.d, nt, tv, Ur, op.U, F, m, n, t, p, partial, s); break;
    }
    {
        const double ent = static_cast<double>(m) * static_cast<double>(n);
        timing_end(tok, s, kSweepF32, ent, ent * sweep_flops_per_entry(op.family, op.d, t, false));
    }
    if (e != hipSuccess) return e;
    return reduce_partials(partial, p.chunks, m, t, op.s2, with_noise ? op.sig2 : 0.0f,
                           with_noise ? Vself : nullptr, out, s);
}

}  // namespace mfgp
