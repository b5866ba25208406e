// FP32 RBF sweep with the squared distances on FP32 MFMA (the Gram form).
//
// The hybrid sweep (hybrid.hip) spends d subtractions and d FMAs per entry on
// the distance, most of its vector-ALU work.  For the RBF kernel, whose entry
// 2^(-r2) is smooth in r2, the squared distance can instead come from
//   r2 = |g_i|^2 + |g_j|^2 - 2 g_i . g_j,     g = u - mean(u),
// with the dot products of a 16 x 16 tile in one v_mfma_f32_16x16x4_f32
// (d <= 4; two for d <= 8).  Translating all points by their mean leaves
// every distance unchanged and keeps the norms small.  The entry is then
// factored,
//   2^(-r2) = 2^(-|g_i|^2) 2^(2 g_i . g_j) 2^(-|g_j|^2),
// the column factor b_j = 2^(-|g_j|^2) is folded into the right-hand sides
// when they are packed (V'_j = b_j V_j) and the row factor a_i into the row's
// sums at the end, so per entry the vector ALU is left only the exp2 of the
// MFMA's 2 g_i . g_j (operand layout in gram_kernels.hpp).  With
// |g|^2 <= kGramMaxNorm = 62 every factor lies in [2^-124, 2^124], inside
// binary32; a factored entry below 2^-126 is an entry below 2^-126.
//
// Accuracy.  The form cancels: r2 carries an absolute rounding error of a
// few ulp of max |g|^2, where the direct differences err relative to r2
// itself.  In a simulation of the FP32 arithmetic the per-column relative
// matvec error against FP64 was 8.8e-7 at max |g|^2 = 30 (N = 1e5, d = 4,
// l = 0.3) and 3.5e-6 at 144 (N = 5e5, d = 2, l = 0.05).  Every launch
// therefore checks max |g|^2 (computed on the device before the sweep, no
// host round trip) against kGramMaxNorm = 62 and, above it, runs the
// direct-difference body of the hybrid sweep on the unscaled fragments
// instead (the packing reads the same maximum and scales only below it).
// An unfactored form for larger norms (the norms as two more MFMA
// dimensions, r2 straight out of the MFMA) met the matvec bar at
// max |g|^2 = 144 (column errors <= 4.7e-6), but its entry errors are
// coherent over a point's row: at N = 5e5 with sigma^2 = 0.01 they moved
// K_y's spectrum by more than sigma^2 and CG diverged, for a sweep only 6%
// faster than direct differences there; it is not built.
// A slightly negative r2 from the cancellation (i ~ j) gives an entry a few
// ulp above 1: within the same error, so r2 is not clamped.
//
// The operator is symmetric up to the rounding of the two factors: the
// exponent of (i, j) and (j, i) is the same sum of the products
// (-2 g_j[k]) g_i[k] = (-2 g_i[k]) g_j[k] (the factor 2 is exact), while a_i
// and b_j are applied on different sides (about one ulp per entry).
#include <algorithm>

#include "gram_kernels.hpp"
#include "internal.hpp"

namespace mfgp {

namespace {

constexpr int kMeanBlocks = 64;

// Per-block column sums of U [n][d] over a contiguous row range (FP64).
__global__ __launch_bounds__(256) void gram_mean_stage1(const float* __restrict__ U, int64_t n, int d,
                                                        double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    for (int k = 0; k < d; ++k) {
        double acc = 0.0;
        for (int64_t j = r0 + threadIdx.x; j < r1; j += 256) acc += static_cast<double>(U[j * d + k]);
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * MFGP_MAX_D + k] = red[0];
        __syncthreads();
    }
}

// mu[k] = mean of column k (fixed order over the block sums); clears the
// running maximum of the norms.
__global__ void gram_mean_stage2(const double* __restrict__ part, int nb, int d, int64_t n,
                                 float* __restrict__ mu, unsigned* __restrict__ gmax) {
    const int k = threadIdx.x;
    if (k < d) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b * MFGP_MAX_D + k];
        mu[k] = static_cast<float>(s / static_cast<double>(n));
    }
    if (k == 0) *gmax = 0u;
}

// G[j] = -2 (u_j - mu) zero-padded to DG, nrm[j] = |u_j - mu|^2, and the
// maximum norm (as the bits of a non-negative float, which order like the
// values) into gmax.  Rows n .. npad - 1 repeat row n - 1, so that the sweeps
// read whole distance tiles without clamping (the V behind them is zero).
template <int DG>
__global__ __launch_bounds__(256) void gram_prep_kernel(const float* __restrict__ U, int64_t n, int64_t npad,
                                                        int d, const float* __restrict__ mu, float* __restrict__ G,
                                                        float* __restrict__ nrm, unsigned* __restrict__ gmax) {
    __shared__ float red[256];
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    float nj = 0.0f;
    if (j < npad) {
        const int64_t js = j < n ? j : n - 1;
#pragma unroll
        for (int k = 0; k < DG; ++k) {
            const float g = k < d ? U[js * d + k] - mu[k] : 0.0f;
            nj = fmaf(g, g, nj);
            G[j * DG + k] = -2.0f * g;
        }
        nrm[j] = nj;
    }
    red[threadIdx.x] = nj;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(gmax, __float_as_uint(red[0]));
}

// Fragments of the hybrid sweep (step q, lane l: V[4 q + l / 16][...]) with
// |g_j|^2 behind them; steps cover j < n rounded up to 16.  While the launch
// takes the Gram branch (max |g|^2 <= kGramMaxNorm, the test the sweep makes)
// the values carry the column factor 2^(-|g_j|^2); otherwise they are V itself
// for the direct-difference branch.
__global__ void pack_gfrag_kernel(const float* __restrict__ V, const float* __restrict__ nrm,
                                  const unsigned* __restrict__ gmax, int64_t n, int t, int nt, int tv,
                                  int64_t nsteps, float* __restrict__ F) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int WS = nt + tv + 1;
    if (idx >= nsteps * 64 * WS) return;
    const int w = static_cast<int>(idx % WS);
    const int64_t lq = idx / WS;
    const int l = static_cast<int>(lq % 64);
    const int64_t q = lq / 64;
    const int64_t j = q * kHK + l / 16;
    const float nj = nrm[j < n ? j : n - 1];
    if (w < nt + tv) {
        const int c = w < nt ? tv + 16 * w + (l % 16) : w - nt;
        const float b = __uint_as_float(*gmax) <= kGramMaxNorm ? __builtin_amdgcn_exp2f(-nj) : 1.0f;
        F[idx] = (j < n) ? V[j * t + c] * b : 0.0f;
    } else {
        F[idx] = nj;
    }
}

// Fragments of the fused two-term sweep: the values and |g_j|^2 of both terms.
__global__ void pack_gfrag2_kernel(const float* __restrict__ V, const float* __restrict__ nrmA,
                                   const float* __restrict__ nrmB, int64_t n, int t, int nt, int tv, int64_t nsteps,
                                   float* __restrict__ F) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int WS = nt + tv + 2;
    if (idx >= nsteps * 64 * WS) return;
    const int w = static_cast<int>(idx % WS);
    const int64_t lq = idx / WS;
    const int l = static_cast<int>(lq % 64);
    const int64_t q = lq / 64;
    const int64_t j = q * kHK + l / 16;
    const int64_t js = j < n ? j : n - 1;
    if (w < nt + tv) {
        const int c = w < nt ? tv + 16 * w + (l % 16) : w - nt;
        F[idx] = (j < n) ? V[j * t + c] : 0.0f;
    } else {
        F[idx] = w == nt + tv ? nrmA[js] : nrmB[js];
    }
}

template <int DGA, int DGB, int NT, int TV>
__global__ __launch_bounds__(kBlock) void sweep_gram2_kernel(
    const float* __restrict__ Ga, const float* __restrict__ nrmA, const unsigned* __restrict__ gmaxA,
    const float* __restrict__ Gb, const float* __restrict__ nrmB, const unsigned* __restrict__ gmaxB,
    const float* __restrict__ Ua, int da, const float* __restrict__ Ub, int db, float rb, const float* __restrict__ F,
    int64_t n, int t, int chunks, int64_t jchunk, float* __restrict__ partial) {
    int rb_, ch;
    map_block(blockIdx.x, chunks, rb_, ch);
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;   // multiple of 16
    const int64_t rbase = static_cast<int64_t>(rb_) * kBlock;
    float* out = partial + static_cast<int64_t>(ch) * n * t + rbase * t;
    if (__uint_as_float(*gmaxA) <= kGramMaxNorm && __uint_as_float(*gmaxB) <= kGramMaxNorm)
        gram2_block<DGA, DGB, NT, TV, true>(Ga, nrmA, Gb, nrmB, Ua, da, Ub, db, rb, F, n, t, rbase, j0, j0 + jchunk,
                                            out);
    else
        gram2_block<DGA, DGB, NT, TV, false>(Ga, nrmA, Gb, nrmB, Ua, da, Ub, db, rb, F, n, t, rbase, j0, j0 + jchunk,
                                             out);
}

template <int D, int NT, int TV>
__global__ __launch_bounds__(kBlock) void sweep_gram_kernel(const float* __restrict__ U, const float* __restrict__ G,
                                                            const float* __restrict__ nrm,
                                                            const unsigned* __restrict__ gmax,
                                                            const float* __restrict__ F, int64_t n, int t,
                                                            int chunks, int64_t jchunk, float* __restrict__ partial) {
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;   // multiple of 16
    const int64_t rbase = static_cast<int64_t>(rb) * kBlock;
    float* out = partial + static_cast<int64_t>(ch) * n * t + rbase * t;
    if (__uint_as_float(*gmax) <= kGramMaxNorm)
        gram_block<D <= 4 ? 4 : 8, NT, TV>(G, nrm, F, n, t, rbase, j0, j0 + jchunk, out);
    else
        hyb_block<MFGP_RBF, D, NT, TV, NT + TV + 1>(U, U, F, n, n, t, rbase, j0, j0 + jchunk, out);
}

bool gram_shape(int t, int& nt, int& tv) {
    if (t == 1) {
        nt = 0;
        tv = 1;
        return true;
    }
    nt = t / 16;
    tv = t % 16;
    return nt >= 1 && nt <= 4 && tv <= 1;
}

SweepPlan plan_gram(int64_t n, int64_t target = 4096) {
    SweepPlan p = plan_sweep(n, n, target);
    p.jchunk = (p.jchunk + kGJ - 1) / kGJ * kGJ;
    return p;
}

// Blocks per launch of the single-term sweep: with one right-hand side a
// block is short (59 VGPRs, 8 resident blocks per CU) and finer j-ranges
// even out the last dispatch round (N = 1e5: 16 -> 32 chunks, 1.51 -> 1.48 ms
// per sweep, 1.58 -> 1.55 ms per call); with more columns the partial sums
// the extra chunks write cost what the balance gains.
int64_t gram_target(int t) { return t == 1 ? 12288 : 4096; }

struct GramLayout {
    size_t frag, part, prep, total;
};

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Preparation region: G [n][8], nrm [n], column-mean partials, mu, gmax.
struct PrepLayout {
    size_t g, nrm, mpart, mu, gmax, total;
};

// Rows of the preparation arrays: n rounded up to 64 (whole distance tiles).
int64_t prep_rows(int64_t n) { return (n + 63) / 64 * 64; }

PrepLayout prep_layout(int64_t n) {
    n = prep_rows(n);
    PrepLayout L{};
    size_t off = 0;
    L.g = off;
    off += up256(static_cast<size_t>(n) * 8 * sizeof(float));
    L.nrm = off;
    off += up256(static_cast<size_t>(n) * sizeof(float));
    L.mpart = off;
    off += up256(static_cast<size_t>(kMeanBlocks) * MFGP_MAX_D * sizeof(double));
    L.mu = off;
    off += 256;
    L.gmax = off;
    off += 256;
    L.total = off;
    return L;
}

GramLayout gram_layout(int64_t n, int t) {
    int nt = 0, tv = 0;
    gram_shape(t, nt, tv);
    const SweepPlan p = plan_gram(n, gram_target(t));
    const SweepPlan p1 = plan_gram(n, gram_target(1));
    const int64_t nsteps = (n + kGJ - 1) / kGJ * (kGJ / kHK);
    GramLayout L{};
    size_t off = 0;
    L.frag = off;
    off += up256(static_cast<size_t>(nsteps) * 64 * (nt + tv + 1) * sizeof(float));
    L.part = off;
    // room for the one-column plan's partials too, so that a workspace sized
    // for t columns also serves every product of fewer columns
    off += up256(std::max(static_cast<size_t>(p.chunks) * n * t, static_cast<size_t>(p1.chunks) * n) * sizeof(float));
    L.prep = off;
    off += prep_layout(n).total;
    L.total = off;
    return L;
}

GramLayout gram2_layout(int64_t n, int t) {
    int nt = 0, tv = 0;
    gram_shape(t, nt, tv);
    const SweepPlan p = plan_gram(n);
    const int64_t nsteps = (n + kGJ - 1) / kGJ * (kGJ / kHK);
    GramLayout L{};
    size_t off = 0;
    L.frag = off;
    off += up256(static_cast<size_t>(nsteps) * 64 * (nt + tv + 2) * sizeof(float));
    L.part = off;
    off += up256(static_cast<size_t>(p.chunks) * n * t * sizeof(float));
    L.prep = off;
    off += 2 * prep_layout(n).total;
    L.total = off;
    return L;
}

template <int DGA, int DGB>
hipError_t launch_gram2_dd(int nt, int tv, const GramPrep& a, const GramPrep& b, const float* Ua, int da,
                           const float* Ub, int db, float rb, const float* F, int64_t n, int t, const SweepPlan& p,
                           float* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
#define MFGP_GRAM2_CASE(NTV, TVV)                                                                             \
    if (nt == NTV && tv == TVV) {                                                                             \
        hipLaunchKernelGGL((sweep_gram2_kernel<DGA, DGB, NTV, TVV>), grid, dim3(kBlock), 0, s, a.G, a.nrm, a.gmax, \
                           b.G, b.nrm, b.gmax, Ua, da, Ub, db, rb, F, n, t, p.chunks, p.jchunk, partial);        \
        return hipGetLastError();                                                                             \
    }
    MFGP_GRAM2_CASE(0, 1)
    MFGP_GRAM2_CASE(1, 0) MFGP_GRAM2_CASE(1, 1) MFGP_GRAM2_CASE(2, 0) MFGP_GRAM2_CASE(2, 1)
    MFGP_GRAM2_CASE(3, 0) MFGP_GRAM2_CASE(3, 1) MFGP_GRAM2_CASE(4, 0) MFGP_GRAM2_CASE(4, 1)
#undef MFGP_GRAM2_CASE
    return hipErrorInvalidValue;
}

template <int D>
hipError_t launch_gram_d(int nt, int tv, const float* U, const float* G, const float* nrm, const unsigned* gmax,
                         const float* F, int64_t n, int t, const SweepPlan& p, float* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
#define MFGP_GRAM_CASE(NTV, TVV)                                                                        \
    if (nt == NTV && tv == TVV) {                                                                       \
        hipLaunchKernelGGL((sweep_gram_kernel<D, NTV, TVV>), grid, dim3(kBlock), 0, s, U, G, nrm, gmax, F, \
                           n, t, p.chunks, p.jchunk, partial);                                          \
        return hipGetLastError();                                                                       \
    }
    MFGP_GRAM_CASE(0, 1)
    MFGP_GRAM_CASE(1, 0) MFGP_GRAM_CASE(1, 1) MFGP_GRAM_CASE(2, 0) MFGP_GRAM_CASE(2, 1)
    MFGP_GRAM_CASE(3, 0) MFGP_GRAM_CASE(3, 1) MFGP_GRAM_CASE(4, 0) MFGP_GRAM_CASE(4, 1)
#undef MFGP_GRAM_CASE
    return hipErrorInvalidValue;
}

}  // namespace

bool gram_supported(int t) {
    int nt, tv;
    return gram_shape(t, nt, tv);
}

size_t gram_scratch_bytes(int64_t n, int t) {
    if (!gram_supported(t)) return 0;
    return gram_layout(n, t).total + 1024;
}

size_t gram_prep_bytes(int64_t n) { return prep_layout(n).total; }

size_t gram2_scratch_bytes(int64_t n, int t) {
    if (!gram_supported(t)) return 0;
    return gram2_layout(n, t).total + 1024;
}

hipError_t gram_prepare(const Operator& op, void* scratch, GramPrep& g, hipStream_t s) {
    const int64_t n = op.n;
    if (op.d < 1 || op.d > 8) return hipErrorNotSupported;
    const PrepLayout L = prep_layout(n);
    char* base = static_cast<char*>(scratch);
    g.G = reinterpret_cast<float*>(base + L.g);
    g.nrm = reinterpret_cast<float*>(base + L.nrm);
    g.gmax = reinterpret_cast<unsigned*>(base + L.gmax);
    g.dg = op.d <= 4 ? 4 : 8;
    return gram_prepare_into(op, g, base + L.mpart, s);
}

size_t gram_mean_bytes() { return static_cast<size_t>(kMeanBlocks) * MFGP_MAX_D * sizeof(double) + 256; }

hipError_t gram_prepare_into(const Operator& op, const GramPrep& g, void* mean_scratch, hipStream_t s) {
    const int64_t n = op.n;
    if (op.d < 1 || op.d > 8) return hipErrorNotSupported;
    double* mpart = static_cast<double*>(mean_scratch);
    float* mu = reinterpret_cast<float*>(mpart + kMeanBlocks * MFGP_MAX_D);
    const int nb = static_cast<int>(std::min<int64_t>(kMeanBlocks, (n + 255) / 256));
    hipLaunchKernelGGL(gram_mean_stage1, dim3(nb), dim3(256), 0, s, op.U, n, op.d, mpart);
    hipLaunchKernelGGL(gram_mean_stage2, dim3(1), dim3(64), 0, s, mpart, nb, op.d, n, mu, g.gmax);
    const int64_t npad = prep_rows(n);
    const unsigned pblocks = static_cast<unsigned>((npad + 255) / 256);
    if (g.dg == 4)
        hipLaunchKernelGGL(gram_prep_kernel<4>, dim3(pblocks), dim3(256), 0, s, op.U, n, npad, op.d, mu, g.G, g.nrm,
                           g.gmax);
    else
        hipLaunchKernelGGL(gram_prep_kernel<8>, dim3(pblocks), dim3(256), 0, s, op.U, n, npad, op.d, mu, g.G, g.nrm,
                           g.gmax);
    return hipGetLastError();
}

hipError_t reduce_partials(const float* partial, int chunks, int64_t m, int t, float s2,
                           float sig2, const float* Vself, float* out, hipStream_t s);

hipError_t apply_gram(const Operator& op, const float* V, int t, float* out, bool with_noise, const float* Vself,
                      void* scratch, hipStream_t s) {
    int nt, tv;
    if (op.family != MFGP_RBF || op.d < 1 || op.d > 8 || !gram_shape(t, nt, tv)) return hipErrorNotSupported;
    const int64_t n = op.n;
    const SweepPlan p = plan_gram(n, gram_target(t));
    const GramLayout L = gram_layout(n, t);
    char* base = static_cast<char*>(scratch);
    float* F = reinterpret_cast<float*>(base + L.frag);
    float* partial = reinterpret_cast<float*>(base + L.part);
    GramPrep gp;
    hipError_t e = hipSuccess;
    if (op.gram_pre)
        gp = *op.gram_pre;   // prepared once by the solver
    else
        e = gram_prepare(op, base + L.prep, gp, s);
    if (e != hipSuccess) return e;
    float* G = gp.G;
    float* nrm = gp.nrm;
    unsigned* gmax = gp.gmax;
    const int64_t nsteps = (n + kGJ - 1) / kGJ * (kGJ / kHK);
    const int64_t total = nsteps * 64 * (nt + tv + 1);
    hipLaunchKernelGGL(pack_gfrag_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, V, nrm,
                       gmax, n, t, nt, tv, nsteps, F);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* tok = timing_begin(s);
    switch (op.d) {
        case 1: e = launch_gram_d<1>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
        case 2: e = launch_gram_d<2>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
        case 3: e = launch_gram_d<3>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
        case 4: e = launch_gram_d<4>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
        case 5: e = launch_gram_d<5>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
        case 6: e = launch_gram_d<6>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
        case 7: e = launch_gram_d<7>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
        default: e = launch_gram_d<8>(nt, tv, op.U, G, nrm, gmax, F, n, t, p, partial, s); break;
    }
    {
        const double ent = static_cast<double>(n) * static_cast<double>(n);
        timing_end(tok, s, kSweepF32, ent, ent * sweep_flops_per_entry(op.family, op.d, t, false));
    }
    if (e != hipSuccess) return e;
    return reduce_partials(partial, p.chunks, n, t, op.s2, with_noise ? op.sig2 : 0.0f, with_noise ? Vself : nullptr,
                           out, s);
}

// The fused sweep of a two-term sum s2_a k_a + s2_b k_b of RBF-class terms
// (RBF, periodic or products of them, each on its own prescaled features):
// both preparations, fragments with both norms, one sweep whose entries are
// k_a + (s2_b / s2_a) k_b, and the reduction with s2_a (and the head's noise).
hipError_t apply_gram2(const Operator& a, const Operator& b, const float* V, int t, float* out, bool with_noise,
                       const float* Vself, void* scratch, hipStream_t s) {
    int nt, tv;
    if (a.family != MFGP_RBF || b.family != MFGP_RBF || a.d < 1 || a.d > 8 || b.d < 1 || b.d > 8 || a.n != b.n ||
        !gram_shape(t, nt, tv))
        return hipErrorNotSupported;
    const int64_t n = a.n;
    const SweepPlan p = plan_gram(n);
    const GramLayout L = gram2_layout(n, t);
    const size_t prep = prep_layout(n).total;
    char* base = static_cast<char*>(scratch);
    float* F = reinterpret_cast<float*>(base + L.frag);
    float* partial = reinterpret_cast<float*>(base + L.part);
    GramPrep ga, gb;
    hipError_t e = gram_prepare(a, base + L.prep, ga, s);
    if (e == hipSuccess) e = gram_prepare(b, base + L.prep + prep, gb, s);
    if (e != hipSuccess) return e;
    const int64_t nsteps = (n + kGJ - 1) / kGJ * (kGJ / kHK);
    const int64_t total = nsteps * 64 * (nt + tv + 2);
    hipLaunchKernelGGL(pack_gfrag2_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, V,
                       ga.nrm, gb.nrm, n, t, nt, tv, nsteps, F);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float rb = static_cast<float>(static_cast<double>(b.s2) / static_cast<double>(a.s2));
    void* tok = timing_begin(s);
    if (ga.dg == 4 && gb.dg == 4)
        e = launch_gram2_dd<4, 4>(nt, tv, ga, gb, a.U, a.d, b.U, b.d, rb, F, n, t, p, partial, s);
    else if (ga.dg == 4)
        e = launch_gram2_dd<4, 8>(nt, tv, ga, gb, a.U, a.d, b.U, b.d, rb, F, n, t, p, partial, s);
    else if (gb.dg == 4)
        e = launch_gram2_dd<8, 4>(nt, tv, ga, gb, a.U, a.d, b.U, b.d, rb, F, n, t, p, partial, s);
    else
        e = launch_gram2_dd<8, 8>(nt, tv, ga, gb, a.U, a.d, b.U, b.d, rb, F, n, t, p, partial, s);
    {
        const double ent = static_cast<double>(n) * static_cast<double>(n);
        timing_end(tok, s, kSweepF32, ent,
                   ent * (sweep_flops_per_entry(a.family, a.d, t, false) + 3.0 * b.d + 2.0));
    }
    if (e != hipSuccess) return e;
    return reduce_partials(partial, p.chunks, n, t, a.s2, with_noise ? a.sig2 : 0.0f, with_noise ? Vself : nullptr,
                           out, s);
}

}  // namespace mfgp
