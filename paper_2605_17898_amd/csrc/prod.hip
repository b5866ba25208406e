// General kernel products: the `*` composition of LightGP Sec. 3 "Kernels"
// over any of its concrete families, s2 prod_f k_f, when a factor is Matern
// or Linear.  (Products of RBF and periodic factors alone are RBF on the
// concatenated features and run every RBF product form; see make_product.)
//
// Features (prescaled once per point, see common.hpp): the RBF-class ones
// first -- the periodic factor's circle features, then each RBF factor's
// x c_RBF / l -- in [0, nr), then for each Matern-nu factor x c_nu / l and for
// each Linear factor x itself, each in its own range [f0, f1).  With
// du = u_i - u_j the unit-scale entry is
//     prod_Matern P_nu(q_f)  prod_Linear (u_i . u_j)_f  2^-(|du|^2_[0,nr) + sum_Matern q_f),
// q_f = |du| over the factor's range, P the Matern polynomial in q_f
// (2^-q = e^(-sqrt(2 nu) rho)): one exp2 per entry for all factors.
//
// Gradient (the adjoint sums, as in adjoint.hip): with k^ the unit-scale
// entry and W_ij = sum_c w_c A_ic B_jc,
//     G_k  = sum W k^ r_f(q_f) du_k^2      per feature k of an RBF-class
//            (r = 1) or Matern factor (r = 1/q, 1/P, (1 + q ln2)/P for
//            nu = 1/2, 3/2, 5/2: the factor's d log g / d l over the RBF
//            form's), 0 for Linear features,
//     G_s  = sum W k^,
//     G_p  = sum W k^ sum_k dx_k (u_i,2k+1 u_j,2k - u_i,2k u_j,2k+1)   (periodic factor),
// and the host applies s2 F_k(l_k) per lengthscale as for the single
// families (Linear factors carry no parameter inside a product).  The sweeps
// are the plain VALU form (one lane per row, wave-uniform j), FP32 entries
// with FP32 two-level or FP64 accumulation, fixed-order reductions.
#include "internal.hpp"
#include "adjoint_kernels.hpp"

#include <cmath>

namespace mfgp {
namespace {

__device__ __forceinline__ float matern_poly(int kind, float q) {
    if (kind == MFGP_MATERN32) return fmaf(q, kLn2, 1.0f);
    if (kind == MFGP_MATERN52) return fmaf(fmaf(q, kLn2Sq3, kLn2), q, 1.0f);
    return 1.0f;
}

// r_f(q) of the file comment from the factor's polynomial value.
__device__ __forceinline__ float matern_ratio(int kind, float q, float poly) {
    if (kind == MFGP_MATERN12) return q > 0.0f ? __builtin_amdgcn_rcpf(q) : 0.0f;
    if (kind == MFGP_MATERN32) return __builtin_amdgcn_rcpf(poly);
    return fmaf(q, kLn2, 1.0f) * __builtin_amdgcn_rcpf(poly);
}

// Unit-scale entry; sq[k] = du_k^2 and, per special factor, q[f] and the
// polynomial value poly[f] (Matern) are left for the adjoint.
template <int D>
__device__ __forceinline__ float prod_entry_full(const float (&ui)[D], const float* __restrict__ uj,
                                                 const ProdDesc& pd, float (&sq)[D], float (&q)[MFGP_MAX_TERMS],
                                                 float (&poly)[MFGP_MAX_TERMS]) {
    float pr[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float df = ui[k] - uj[k];
        sq[k] = df * df;
        pr[k] = ui[k] * uj[k];
    }
    float e = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) e += k < pd.nr ? sq[k] : 0.0f;
    float mult = 1.0f;
#pragma unroll
    for (int f = 0; f < MFGP_MAX_TERMS; ++f) {
        q[f] = 0.0f;
        poly[f] = 1.0f;
        if (f < pd.nspec) {
            const bool lin = pd.kind[f] == MFGP_LINEAR;
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const bool in = k >= pd.f0[f] && k < pd.f1[f];
                s += in ? (lin ? pr[k] : sq[k]) : 0.0f;
            }
            if (lin) {
                mult *= s;
            } else {
                q[f] = __builtin_amdgcn_sqrtf(s);
                e += q[f];
                poly[f] = matern_poly(pd.kind[f], q[f]);
                mult *= poly[f];
            }
        }
    }
    return mult * __builtin_amdgcn_exp2f(-e);
}

template <int D>
__device__ __forceinline__ float prod_entry(const float (&ui)[D], const float* __restrict__ uj, const ProdDesc& pd) {
    float sq[D], q[MFGP_MAX_TERMS], poly[MFGP_MAX_TERMS];
    return prod_entry_full<D>(ui, uj, pd, sq, q, poly);
}

template <int D, int TB>
__global__ __launch_bounds__(kBlock) void sweep_prod_kernel(const float* __restrict__ Ur, const float* __restrict__ Uc,
                                                            const float* __restrict__ V, int64_t m, int64_t n,
                                                            int chunks, int64_t jchunk, float* __restrict__ partial,
                                                            ProdDesc pd) {
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t i = static_cast<int64_t>(rb) * kBlock + threadIdx.x;
    const int64_t ii = i < m ? i : m - 1;
    float ui[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ui[k] = Ur[ii * D + k];
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;
    const int64_t jend = j0 + jchunk < n ? j0 + jchunk : n;
    const int cnt = j0 < jend ? static_cast<int>(jend - j0) : 0;
    const float* uc = Uc + j0 * D;
    const float* vc = V + j0 * TB;
    // two-level FP32 accumulation over segments of kSeg j, as the other sweeps
    float acc[TB], tot[TB];
#pragma unroll
    for (int c = 0; c < TB; ++c) {
        acc[c] = 0.0f;
        tot[c] = 0.0f;
    }
    for (int q = 0; q < cnt; ++q) {
        if (q % kSeg == 0 && q > 0) {
#pragma unroll
            for (int c = 0; c < TB; ++c) {
                tot[c] += acc[c];
                acc[c] = 0.0f;
            }
        }
        const float e = prod_entry<D>(ui, uc + q * D, pd);
#pragma unroll
        for (int c = 0; c < TB; ++c) acc[c] = fmaf(e, vc[q * TB + c], acc[c]);
    }
    if (i < m) {
        float* p = partial + (static_cast<int64_t>(ch) * m + i) * TB;
#pragma unroll
        for (int c = 0; c < TB; ++c) p[c] = acc[c] + tot[c];
    }
}

// The same entries with FP64 accumulation against FP64 right-hand sides
// (the solver's recomputed residual).
template <int D, int TB>
__global__ __launch_bounds__(kBlock) void sweep_prod_f64_kernel(const float* __restrict__ Ur,
                                                                const float* __restrict__ Uc,
                                                                const double* __restrict__ V, int ldv, int64_t m,
                                                                int64_t n, int chunks, int64_t jchunk,
                                                                double* __restrict__ partial, ProdDesc pd) {
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t i = static_cast<int64_t>(rb) * kBlock + threadIdx.x;
    const int64_t ii = i < m ? i : m - 1;
    float ui[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ui[k] = Ur[ii * D + k];
    double acc[TB];
#pragma unroll
    for (int c = 0; c < TB; ++c) acc[c] = 0.0;
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;
    const int64_t j1 = j0 + jchunk < n ? j0 + jchunk : n;
    for (int64_t j = j0; j < j1; ++j) {
        const double e = static_cast<double>(prod_entry<D>(ui, Uc + j * D, pd));
        const double* vj = V + j * ldv;
#pragma unroll
        for (int c = 0; c < TB; ++c) acc[c] = fma(e, vj[c], acc[c]);
    }
    if (i < m) {
        double* p = partial + (static_cast<int64_t>(ch) * m + i) * TB;
#pragma unroll
        for (int c = 0; c < TB; ++c) p[c] = acc[c];
    }
}

// Adjoint sums [G_0 .. G_{D-1}, G_s, G_p] per block (see the file comment).
// X [n, din] raw inputs (read only when the product has a periodic factor,
// whose circle features are [0, 2 din)).
template <int D, int TB>
__global__ __launch_bounds__(kBlock) void adjoint_prod_kernel(const float* __restrict__ X, int din, int periodic,
                                                              const float* __restrict__ U,
                                                              const float* __restrict__ A, int lda, int c0, ColW w,
                                                              const float* __restrict__ B, int64_t n, int chunks,
                                                              int64_t jchunk, double* __restrict__ partial,
                                                              ProdDesc pd) {
    constexpr int W = D + 2;
    constexpr int kMaxIn = MFGP_MAX_D / 2;   // inputs of a periodic factor
    __shared__ double red[W * (kBlock / 64)];
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t i = static_cast<int64_t>(rb) * kBlock + threadIdx.x;
    const int64_t ii = i < n ? i : n - 1;
    float ui[D], ai[TB], xi[kMaxIn];
#pragma unroll
    for (int k = 0; k < D; ++k) ui[k] = U[ii * D + k];
#pragma unroll
    for (int k = 0; k < kMaxIn; ++k) xi[k] = periodic && k < din ? X[ii * din + k] : 0.0f;
#pragma unroll
    for (int c = 0; c < TB; ++c) ai[c] = i < n ? A[ii * lda + c0 + c] * w.w[c] : 0.0f;
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;
    const int64_t jend = j0 + jchunk < n ? j0 + jchunk : n;
    const int cnt = j0 < jend ? static_cast<int>(jend - j0) : 0;
    const float* uc = U + j0 * D;
    const float* bc = B + j0 * TB;
    float g[W], tg[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        g[k] = 0.0f;
        tg[k] = 0.0f;
    }
    for (int q = 0; q < cnt; ++q) {
        if (q % kSeg == 0 && q > 0) {
#pragma unroll
            for (int k = 0; k < W; ++k) {
                tg[k] += g[k];
                g[k] = 0.0f;
            }
        }
        const float* uj = uc + q * D;
        float sq[D], qf[MFGP_MAX_TERMS], poly[MFGP_MAX_TERMS];
        const float kv = prod_entry_full<D>(ui, uj, pd, sq, qf, poly);
        float wij = 0.0f;
#pragma unroll
        for (int c = 0; c < TB; ++c) wij = fmaf(ai[c], bc[q * TB + c], wij);
        const float wk = wij * kv;
        // per-feature weight: 1 (RBF-class), r_f (Matern), 0 (Linear)
        float wt[D];
#pragma unroll
        for (int k = 0; k < D; ++k) wt[k] = k < pd.nr ? 1.0f : 0.0f;
#pragma unroll
        for (int f = 0; f < MFGP_MAX_TERMS; ++f) {
            if (f < pd.nspec && pd.kind[f] != MFGP_LINEAR) {
                const float r = matern_ratio(pd.kind[f], qf[f], poly[f]);
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (k >= pd.f0[f] && k < pd.f1[f]) wt[k] = r;
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) g[k] = fmaf(wk * wt[k], sq[k], g[k]);
        g[D] += wk;
        if (periodic) {
            float h = 0.0f;
#pragma unroll
            for (int k = 0; k < kMaxIn; ++k) {
                if (2 * k + 1 < D && k < din) {
                    const float cr = fmaf(ui[2 * k + 1], uj[2 * k], -ui[2 * k] * uj[2 * k + 1]);
                    h = fmaf(xi[k] - X[(j0 + q) * din + k], cr, h);
                }
            }
            g[D + 1] = fmaf(wk, h, g[D + 1]);
        }
    }
    double v[W];
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = static_cast<double>(tg[k]) + static_cast<double>(g[k]);
    block_sum_write<W>(v, red, partial + static_cast<int64_t>(blockIdx.x) * W);
}

// var[i] += s2 k^(x_i, x_i) (the Linear factors' |x_i|^2; 1 without them)
template <int D>
__global__ void prod_prior_kernel(const float* __restrict__ Ur, int64_t m, ProdDesc pd, double s2,
                                  float* __restrict__ var) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    float ui[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ui[k] = Ur[i * D + k];
    var[i] = static_cast<float>(static_cast<double>(var[i]) + s2 * static_cast<double>(prod_entry<D>(ui, Ur + i * D, pd)));
}

template <int D>
hipError_t sweep_prod_f32_d(int tb, const SweepArgs& a, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.plan.rowblocks) * a.plan.chunks);
    switch (tb) {
#define MFGP_CASE(TBV)                                                                                          \
    case TBV:                                                                                                   \
        hipLaunchKernelGGL((sweep_prod_kernel<D, TBV>), grid, dim3(kBlock), 0, s, a.Ur, a.Uc, a.V, a.m, a.n,     \
                           a.plan.chunks, a.plan.jchunk, a.partial, *a.pd);                                     \
        return hipGetLastError();
        MFGP_TB_LIST(MFGP_CASE)
#undef MFGP_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int D>
hipError_t sweep_prod_f64_d(int tb, const SweepArgs64& a, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.plan.rowblocks) * a.plan.chunks);
    switch (tb) {
#define MFGP_CASE(TBV)                                                                                            \
    case TBV:                                                                                                     \
        hipLaunchKernelGGL((sweep_prod_f64_kernel<D, TBV>), grid, dim3(kBlock), 0, s, a.Ur, a.Uc, a.V, a.ldv,     \
                           a.m, a.n, a.plan.chunks, a.plan.jchunk, a.partial, *a.pd);                             \
        return hipGetLastError();
        MFGP_TB64_LIST(MFGP_CASE)
#undef MFGP_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int D>
hipError_t adjoint_prod_d(const Operator& op, int tb, const float* A, int lda, int c0, const ColW& w,
                          const float* B, const SweepPlan& p, double* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
    switch (tb) {
#define MFGP_CASE(TBV)                                                                                          \
    case TBV:                                                                                                   \
        hipLaunchKernelGGL((adjoint_prod_kernel<D, TBV>), grid, dim3(kBlock), 0, s, op.X, op.din, op.periodic,   \
                           op.U, A, lda, c0, w, B, op.n, p.chunks, p.jchunk, partial, op.pd);                   \
        return hipGetLastError();
        MFGP_TB_LIST(MFGP_CASE)
#undef MFGP_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

#define MFGP_D_SWITCH(CALL)        \
    switch (D) {                   \
        case 1: return CALL(1);    \
        case 2: return CALL(2);    \
        case 3: return CALL(3);    \
        case 4: return CALL(4);    \
        case 5: return CALL(5);    \
        case 6: return CALL(6);    \
        case 7: return CALL(7);    \
        case 8: return CALL(8);    \
        default: return hipErrorInvalidValue; \
    }

hipError_t sweep_prod_f32(int D, int tb, const SweepArgs& a, hipStream_t s) {
    if (!a.pd) return hipErrorInvalidValue;
#define MFGP_CALL(DV) sweep_prod_f32_d<DV>(tb, a, s)
    MFGP_D_SWITCH(MFGP_CALL)
#undef MFGP_CALL
}

hipError_t sweep_prod_f64(int D, int tb, const SweepArgs64& a, hipStream_t s) {
    if (!a.pd) return hipErrorInvalidValue;
#define MFGP_CALL(DV) sweep_prod_f64_d<DV>(tb, a, s)
    MFGP_D_SWITCH(MFGP_CALL)
#undef MFGP_CALL
}

hipError_t adjoint_prod(const Operator& op, int tb, const float* A, int lda, int c0, const float* w_host,
                        const float* B, const SweepPlan& p, double* partial, hipStream_t s) {
    ColW w{};
    for (int c = 0; c < tb; ++c) w.w[c] = w_host[c];
    const int D = op.d;
#define MFGP_CALL(DV) adjoint_prod_d<DV>(op, tb, A, lda, c0, w, B, p, partial, s)
    MFGP_D_SWITCH(MFGP_CALL)
#undef MFGP_CALL
}

hipError_t prod_prior_add(const Operator& op, const float* Ur, int64_t m, double s2, float* var, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((m + 255) / 256));
    switch (op.d) {
#define MFGP_CASE(DV)                                                                                   \
    case DV:                                                                                            \
        hipLaunchKernelGGL(prod_prior_kernel<DV>, grid, dim3(256), 0, s, Ur, m, op.pd, s2, var);       \
        return hipGetLastError();
        MFGP_CASE(1) MFGP_CASE(2) MFGP_CASE(3) MFGP_CASE(4) MFGP_CASE(5) MFGP_CASE(6) MFGP_CASE(7) MFGP_CASE(8)
#undef MFGP_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mfgp
