// Adjoint sweep: sums over all kernel entries of W_ij dk_ij/dtheta with
// W_ij = sum_c w_c A_ic B_jc, generated per entry and never stored.
//
// It gives the vector-Jacobian product  sum_c w_c A_c^T (dK/dtheta) B_c,
// and with A = [alpha, K_y^{-1} Z], B = [alpha, Z], w = [1/2, -1/(2p), ...]
// the gradient of the log marginal likelihood
//   d/dtheta log p(y|X) = 1/2 alpha^T dK alpha - 1/2 tr(K_y^{-1} dK)
// with the trace replaced by its Rademacher-probe estimate (LightGP Sec. 2,
// the log p(y|X) formula; Sec. 4.3, Hutchinson with Rademacher probes).  The
// paper's own optimiser uses finite differences (Sec. 5); this pass replaces
// the 2P+1 fits by one sweep.
//
// In prescaled coordinates (u = x c / l, see common.hpp) with
// du_k = u_ik - u_jk and q = |u_i - u_j|:
//   d k / d l_k = s2 * F_k * g(q) * du_k^2   with
//   RBF         g = 2^(-q^2)               F_k = 1 / (c^2 l_k)
//   Matern-1/2  g = 2^(-q) / q  (0 at q=0)  F_k = 1 / (c l_k)
//   Matern-3/2  g = 2^(-q)                 F_k = 3 / (c^2 l_k)
//   Matern-5/2  g = (1 + q ln2) 2^(-q)     F_k = (5/3) / (c^2 l_k)
//   d k / d s2  = k^ (unit-outputscale entry)
// The sweep accumulates G_k = sum_ij W_ij g du_k^2 and G_s = sum_ij W_ij k^;
// the host applies s2 F_k.  Lane sums are FP32 over one j-range; block,
// grid and host sums are FP64 in a fixed order.
#include "internal.hpp"
#include "adjoint_kernels.hpp"

namespace mfgp {

template <int FAM, int D, int TB>
__global__ __launch_bounds__(kBlock) void adjoint_kernel(
    const float* __restrict__ U, const float* __restrict__ A, int lda, int c0, ColW w,
    const float* __restrict__ B, int64_t n, int chunks, int64_t jchunk,
    double* __restrict__ partial) {
    // B is a packed [n, TB] block; A is read at columns c0 .. c0+TB-1 of [n, lda].
    __shared__ double red[(D + 1) * (kBlock / 64)];
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t i = static_cast<int64_t>(rb) * kBlock + threadIdx.x;
    const int64_t ii = i < n ? i : n - 1;
    float ui[D], ai[TB];
#pragma unroll
    for (int k = 0; k < D; ++k) ui[k] = U[ii * D + k];
#pragma unroll
    for (int c = 0; c < TB; ++c) ai[c] = i < n ? A[ii * lda + c0 + c] * w.w[c] : 0.0f;
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;
    const int64_t jend = j0 + jchunk < n ? j0 + jchunk : n;
    const int cnt = j0 < jend ? static_cast<int>(jend - j0) : 0;
    double v[D + 1];
    adjoint_rows<FAM, D, TB>(ui, ai, U + j0 * D, B + j0 * TB, cnt, v);
    block_sum_write<D + 1>(v, red, partial + static_cast<int64_t>(blockIdx.x) * (D + 1));
}

// The same sums with the weights W_ij = sum_c (w_c A_ic) B_jc on the FP32
// matrix cores (many right-hand sides: tb >= 16).  Rows as in the product
// sweeps (a wave owns kHRT tiles of 16 rows, a block 256 rows), j in blocks
// of 16.  Per row tile and block, NC = ceil(tb / 4) v_mfma_f32_16x16x4_f32
// contract over the columns c: the A operand (16 j x 4 c) is lane l's
// B[jb + l % 16][4 k + l / 16], the B operand (4 c x 16 i) its
// w_c A[i][4 k + l / 16], so accumulator register s of lane l holds W_ij for
// i = row l % 16 and j = jb + 4 (l / 16) + s; columns c >= tb and rows j past
// the range carry zeros.  The lane then forms that entry's distance, kernel
// value and derivative factor on the VALU (as adjoint_rows) and accumulates
// W_ij g du_k^2 and W_ij k^ in two-level FP32 sums.  The VALU work per entry
// drops from ~(tb + 5d + 4) to ~(5d + 4) operations; the contraction costs
// NC MFMAs per 256 entries.
template <int FAM, int D, int NC>
__global__ __launch_bounds__(kBlock) void adjoint_mfma_kernel(
    const float* __restrict__ U, const float* __restrict__ A, int lda, int c0, ColW w,
    const float* __restrict__ B, int tb, int64_t n, int chunks, int64_t jchunk,
    double* __restrict__ partial) {
    __shared__ double red[(D + 1) * (kBlock / 64)];
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int grp = lane >> 4;
    const int r16 = lane & 15;
    const int64_t row0 = static_cast<int64_t>(rb) * kBlock + wave * (kHRT * 16);

    // B operand (w_c A_ic) and u_i of the lane's row in each row tile
    float ai[kHRT][NC], ui[kHRT][D];
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
        const int64_t i = row0 + r * 16 + r16;
        const int64_t ic = i < n ? i : n - 1;
#pragma unroll
        for (int k = 0; k < D; ++k) ui[r][k] = U[ic * D + k];
#pragma unroll
        for (int kc = 0; kc < NC; ++kc) {
            const int c = 4 * kc + grp;
            ai[r][kc] = (i < n && c < tb) ? A[ic * lda + c0 + c] * w.w[c] : 0.0f;
        }
    }
    float g[kHRT][D], gs[kHRT], tg[kHRT][D], ts[kHRT];
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
        gs[r] = 0.0f;
        ts[r] = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            g[r][k] = 0.0f;
            tg[r][k] = 0.0f;
        }
    }

    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;
    const int64_t j1 = j0 + jchunk < n ? j0 + jchunk : n;
    const int64_t nblk = j0 < j1 ? (j1 - j0 + 15) / 16 : 0;
    const f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t jb = j0 + b * 16;
        // A operand: B rows of the block (zero past the range and past tb)
        const int64_t ja = jb + r16;
        float bj[NC];
#pragma unroll
        for (int kc = 0; kc < NC; ++kc) {
            const int c = 4 * kc + grp;
            bj[kc] = (ja < j1 && c < tb) ? B[ja * tb + c] : 0.0f;
        }
        // u_j of the lane's four entries (clamped rows carry W = 0)
        float uj[4][D];
#pragma unroll
        for (int sq = 0; sq < 4; ++sq) {
            int64_t js = jb + 4 * grp + sq;
            js = js < n ? js : n - 1;
#pragma unroll
            for (int k = 0; k < D; ++k) uj[sq][k] = U[js * D + k];
        }
#pragma unroll
        for (int r = 0; r < kHRT; ++r) {
            f32x4 W = zero4;
#pragma unroll
            for (int kc = 0; kc < NC; ++kc) W = __builtin_amdgcn_mfma_f32_16x16x4f32(bj[kc], ai[r][kc], W, 0, 0, 0);
#pragma unroll
            for (int sq = 0; sq < 4; ++sq) {
                float df[D];
                float d2 = 0.0f;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    df[k] = ui[r][k] - uj[sq][k];
                    d2 = fmaf(df[k], df[k], d2);
                }
                float kv, gf;
                kentry_and_dfac<FAM>(d2, kv, gf);
                const float wij = W[sq];
                gs[r] = fmaf(wij, kv, gs[r]);
                const float wd = wij * gf;
#pragma unroll
                for (int k = 0; k < D; ++k) g[r][k] = fmaf(wd * df[k], df[k], g[r][k]);
            }
        }
        if (((b + 1) & (kSeg / 16 - 1)) == 0) {
#pragma unroll
            for (int r = 0; r < kHRT; ++r) {
                ts[r] += gs[r];
                gs[r] = 0.0f;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    tg[r][k] += g[r][k];
                    g[r][k] = 0.0f;
                }
            }
        }
    }
    double v[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) v[k] = 0.0;
#pragma unroll
    for (int r = 0; r < kHRT; ++r) {
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] += static_cast<double>(tg[r][k]) + static_cast<double>(g[r][k]);
        v[D] += static_cast<double>(ts[r]) + static_cast<double>(gs[r]);
    }
    block_sum_write<D + 1>(v, red, partial + static_cast<int64_t>(blockIdx.x) * (D + 1));
}

// Grid sum of component k (block k) over the sweep's block partials: 256
// threads stride the blocks, then a fixed tree (the same order every call).
__global__ __launch_bounds__(256) void adjoint_final_kernel(const double* __restrict__ partial, int nblocks,
                                                            int width, double* __restrict__ out, int accumulate) {
    __shared__ double lds[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[static_cast<int64_t>(b) * width + k];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = accumulate ? out[k] + lds[0] : lds[0];
}

template <int FAM, int D>
static hipError_t adjoint_fd(int tb, const float* U, const float* A, int lda, int c0,
                             const ColW& w, const float* B, int64_t n, const SweepPlan& p,
                             double* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
    switch (tb) {
        // many right-hand sides: the weights on the matrix cores
#define MFGP_MCASE(TBV, NCV)                                                                          \
    case TBV:                                                                                         \
        hipLaunchKernelGGL((adjoint_mfma_kernel<FAM, D, NCV>), grid, dim3(kBlock), 0, s, U, A, lda, c0, w, \
                           B, TBV, n, p.chunks, p.jchunk, partial);                                   \
        return hipGetLastError();
        MFGP_MCASE(16, 4) MFGP_MCASE(17, 5) MFGP_MCASE(32, 8) MFGP_MCASE(33, 9)
#undef MFGP_MCASE
#define MFGP_CASE(TBV)                                                                        \
    case TBV:                                                                                 \
        hipLaunchKernelGGL((adjoint_kernel<FAM, D, TBV>), grid, dim3(kBlock), 0, s, U, A, lda, \
                           c0, w, B, n, p.chunks, p.jchunk, partial);                         \
        return hipGetLastError();
        MFGP_CASE(1) MFGP_CASE(2) MFGP_CASE(3) MFGP_CASE(4) MFGP_CASE(5) MFGP_CASE(6) MFGP_CASE(7) MFGP_CASE(8)
#undef MFGP_CASE
        default:
            return hipErrorInvalidValue;
    }
}

// Periodic family (RBF on the circle features u = c (cos th, sin th) / l,
// th = 2 pi x / p, see make_operator).  Per entry, with du = u_i - u_j over the
// 2 DIN features and k^ = 2^(-|du|^2):
//   G_l[k] += W_ij k^ (du_2k^2 + du_2k+1^2)   (both features of input k scale with 1/l_k)
//   G_s    += W_ij k^
//   G_p    += W_ij k^ sum_k (x_ik - x_jk) (u_i,2k+1 u_j,2k - u_i,2k u_j,2k+1)
// The last bracket is (c / l_k)^2 sin(th_ik - th_jk), so that
//   dk/dp = s2 k^ sum_k (2 pi (x_ik - x_jk) / (p^2 l_k^2)) sin(2 pi (x_ik - x_jk) / p)
// is s2 (2 pi / (p^2 c^2)) times the G_p term; the host applies the factors.
// A product term with RBF factors carries DEX more features after the 2 DIN
// periodic ones (entries 2^(-|du|^2) over all of them); their per-feature
// sums G_x[q] += W_ij k^ du_q^2 follow G_l.  Output: [G_l (DIN), G_x (DEX),
// G_s, G_p].
template <int DIN, int DEX, int TB>
__global__ __launch_bounds__(kBlock) void adjoint_periodic_kernel(
    const float* __restrict__ X, const float* __restrict__ U, const float* __restrict__ A, int lda, int c0,
    ColW w, const float* __restrict__ B, int64_t n, int chunks, int64_t jchunk, double* __restrict__ partial) {
    constexpr int D = 2 * DIN + DEX;
    constexpr int W = DIN + DEX + 2;
    __shared__ double red[W * (kBlock / 64)];
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t i = static_cast<int64_t>(rb) * kBlock + threadIdx.x;
    const int64_t ii = i < n ? i : n - 1;
    float ui[D], xi[DIN], ai[TB];
#pragma unroll
    for (int k = 0; k < D; ++k) ui[k] = U[ii * D + k];
#pragma unroll
    for (int k = 0; k < DIN; ++k) xi[k] = X[ii * DIN + k];
#pragma unroll
    for (int c = 0; c < TB; ++c) ai[c] = i < n ? A[ii * lda + c0 + c] * w.w[c] : 0.0f;
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;
    const int64_t jend = j0 + jchunk < n ? j0 + jchunk : n;
    const int cnt = j0 < jend ? static_cast<int>(jend - j0) : 0;
    const float* uc = U + j0 * D;
    const float* xc = X + j0 * DIN;
    const float* bc = B + j0 * TB;
    // two-level FP32 sums (kSeg entries per level-one segment), FP64 at the end
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
        float df[D];
        float d2 = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            df[k] = ui[k] - uj[k];
            d2 = fmaf(df[k], df[k], d2);
        }
        const float kv = __builtin_amdgcn_exp2f(-d2);
        float wij = 0.0f;
#pragma unroll
        for (int c = 0; c < TB; ++c) wij = fmaf(ai[c], bc[q * TB + c], wij);
        const float wk = wij * kv;
        float h = 0.0f;
#pragma unroll
        for (int k = 0; k < DIN; ++k) {
            g[k] = fmaf(wk, fmaf(df[2 * k], df[2 * k], df[2 * k + 1] * df[2 * k + 1]), g[k]);
            const float cr = fmaf(ui[2 * k + 1], uj[2 * k], -ui[2 * k] * uj[2 * k + 1]);
            h = fmaf(xi[k] - xc[q * DIN + k], cr, h);
        }
#pragma unroll
        for (int e = 0; e < DEX; ++e) g[DIN + e] = fmaf(wk * df[2 * DIN + e], df[2 * DIN + e], g[DIN + e]);
        g[DIN + DEX] += wk;
        g[DIN + DEX + 1] = fmaf(wk, h, g[DIN + DEX + 1]);
    }
    double v[W];
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = static_cast<double>(tg[k]) + static_cast<double>(g[k]);
    block_sum_write<W>(v, red, partial + static_cast<int64_t>(blockIdx.x) * W);
}

template <int DIN, int DEX>
static hipError_t adjoint_periodic_d(int tb, const float* X, const float* U, const float* A, int lda, int c0,
                                     const ColW& w, const float* B, int64_t n, const SweepPlan& p,
                                     double* partial, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(p.rowblocks) * p.chunks);
    switch (tb) {
#define MFGP_CASE(TBV)                                                                                         \
    case TBV:                                                                                                  \
        hipLaunchKernelGGL((adjoint_periodic_kernel<DIN, DEX, TBV>), grid, dim3(kBlock), 0, s, X, U, A, lda, c0, \
                           w, B, n, p.chunks, p.jchunk, partial);                                             \
        return hipGetLastError();
        MFGP_TB_LIST(MFGP_CASE)
#undef MFGP_CASE
        default:
            return hipErrorInvalidValue;
    }
}

// (DIN, DEX): the periodic term alone (DEX = 0) and the products with up to
// three RBF factors of DIN features each within MFGP_MAX_D features.
static hipError_t adjoint_periodic(int din, int dex, int tb, const float* X, const float* U, const float* A,
                                   int lda, int c0, const ColW& w, const float* B, int64_t n, const SweepPlan& p,
                                   double* partial, hipStream_t s) {
#define MFGP_PD(DI, DE) \
    if (din == DI && dex == DE) return adjoint_periodic_d<DI, DE>(tb, X, U, A, lda, c0, w, B, n, p, partial, s);
    MFGP_PD(1, 0)
    MFGP_PD(1, 1)
    MFGP_PD(1, 2)
    MFGP_PD(1, 3)
    MFGP_PD(2, 0)
    MFGP_PD(2, 2)
    MFGP_PD(2, 4)
    MFGP_PD(3, 0)
    MFGP_PD(4, 0)
#undef MFGP_PD
    return hipErrorInvalidValue;
}

template <int FAM>
static hipError_t adjoint_f(int D, int tb, const float* U, const float* A, int lda, int c0,
                            const ColW& w, const float* B, int64_t n, const SweepPlan& p,
                            double* partial, hipStream_t s) {
    switch (D) {
        case 1: return adjoint_fd<FAM, 1>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        case 2: return adjoint_fd<FAM, 2>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        case 3: return adjoint_fd<FAM, 3>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        case 4: return adjoint_fd<FAM, 4>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        case 5: return adjoint_fd<FAM, 5>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        case 6: return adjoint_fd<FAM, 6>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        case 7: return adjoint_fd<FAM, 7>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        case 8: return adjoint_fd<FAM, 8>(tb, U, A, lda, c0, w, B, n, p, partial, s);
        default: return hipErrorInvalidValue;
    }
}

// Per-block partial width: d + 1 sums for the single families, at most
// d + 2 (a general product: per feature, G_s, G_p).
size_t adjoint_scratch_doubles(int64_t n, int d, int t) {
    const SweepPlan p = plan_sweep(n, n);
    const size_t part = static_cast<size_t>(p.rowblocks) * p.chunks * (d + 2);
    const int tb = column_block(t);
    const size_t pack = tb == t ? 0 : (static_cast<size_t>(n) * tb + 1) / 2 + 64;
    return part + pack + 2 * (d + 2) + 128;
}

// sums_host[0..d-1] = G_k, sums_host[d] = G_s (see the file comment); for the
// periodic family (alone or in a product) sums_host[0..din-1] = G_l, then the
// dextra G_x, then G_s, G_p (see adjoint_periodic_kernel).
hipError_t adjoint_sums(const Operator& op, const float* A, const float* B, int t,
                        const double* colw_host, double* sums_host, double* scratch,
                        hipStream_t s) {
    const int d = op.d;
    const int width = op.general ? d + 2 : (op.periodic ? op.din + op.dextra + 2 : d + 1);
    const int64_t n = op.n;
    const SweepPlan p = plan_sweep(n, n);
    const int nblocks = p.rowblocks * p.chunks;
    double* partial = scratch;
    double* total = scratch + static_cast<size_t>(nblocks) * (d + 2) + 64;
    float* pack = reinterpret_cast<float*>(total + 2 * (d + 2) + 64);
    int first = 1;
    for (int c0 = 0; c0 < t;) {
        const int tb = column_block(t - c0);
        ColW w{};
        for (int c = 0; c < tb; ++c) w.w[c] = static_cast<float>(colw_host[c0 + c]);
        const float* bb = B;
        if (tb != t) {
            hipError_t e = launch_pack_cols(B, t, c0, tb, n, pack, s);
            if (e != hipSuccess) return e;
            bb = pack;
        }
        hipError_t e;
        void* tok = timing_begin(s);
        if (op.general) {
            e = adjoint_prod(op, tb, A, t, c0, w.w, bb, p, partial, s);
        } else if (op.periodic) {
            e = adjoint_periodic(op.din, op.dextra, tb, op.X, op.U, A, t, c0, w, bb, n, p, partial, s);
        } else switch (op.family) {
            case MFGP_RBF: e = adjoint_f<MFGP_RBF>(d, tb, op.U, A, t, c0, w, bb, n, p, partial, s); break;
            case MFGP_MATERN12: e = adjoint_f<MFGP_MATERN12>(d, tb, op.U, A, t, c0, w, bb, n, p, partial, s); break;
            case MFGP_MATERN32: e = adjoint_f<MFGP_MATERN32>(d, tb, op.U, A, t, c0, w, bb, n, p, partial, s); break;
            default: e = adjoint_f<MFGP_MATERN52>(d, tb, op.U, A, t, c0, w, bb, n, p, partial, s); break;
        }
        {
            const double ent = static_cast<double>(n) * static_cast<double>(n);
            timing_end(tok, s, kSweepAdjoint, ent, ent * sweep_flops_per_entry(op.family, d, tb, true));
        }
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(adjoint_final_kernel, dim3(width), dim3(256), 0, s, partial, nblocks, width,
                           total, first ? 0 : 1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        first = 0;
        c0 += tb;
    }
    hipError_t e = hipMemcpyAsync(sums_host, total, width * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

}  // namespace mfgp
