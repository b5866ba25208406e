// Batched GP problems: many uneven problems solved together (LightGP Sec. 5
// names batched solves among the CG features its plain loop lacks).
//
// * One persistent launch per product.  The work of all problems is a queue
//   of tiles (problem b, 256-row block, j-range), sorted longest first; the
//   resident workgroups pull tiles through an atomic counter until the queue
//   is empty (every workgroup exits when the counter passes the end), and each
//   tile writes its partial sums to its own slot, reduced afterwards in a
//   fixed order -- so results do not depend on which workgroup took which tile.
// * Per-problem CG on packed [sum n_b, t] blocks: reductions are segmented
//   (each block of the reduction kernels owns rows of one problem only).
// * The iterations between host convergence checks are captured once into a
//   hipGraph and replayed (no memset nodes: the queue counter is reset by a
//   kernel).
// * The tile j-length is picked by timing candidate lengths on the batch
//   itself (plan autotuner) and kept in the plan.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "stall.hpp"
#include "adjoint_kernels.hpp"
#include "cg.hpp"
#include "hybrid_kernels.hpp"
#include "mfma_kernels.hpp"
#include "internal.hpp"

int mfgp_slq_quadrature(const double* coeffs, int32_t m, double znorm2, double* q);

namespace mfgp {

struct BProb {
    int64_t n;          // rows
    int64_t row_off;    // first packed row
    int64_t u_off;      // element offset of U_b (= x_off)
    int64_t jchunk;     // j-range length of this problem's tiles (a multiple of 4)
    int64_t f_off;      // float offset of this problem's FP32-MFMA fragments of V
    int64_t g_off;      // bf16x8 offset of this problem's BF16 fragments of V
    int64_t y_off;      // float offset of this problem's FP32 column-0 copy
    int d;
    int chunks;         // j-ranges per row block
    int tile_base;      // first tile id of this problem
    int rowblocks;
    float s2;
    float sig2;
};
struct BTile {
    int b, rb, ch, id;
};
struct BSeg {
    int b;
    int pad;
    int64_t r0, r1;     // packed rows [r0, r1) of problem b
};

constexpr int kSegRows = 2048;
// Residual replacement keeps the direction only while |r_true - r_rec|^2 <=
// 1e-2 |r_true|^2 (as in the single-problem solver).
constexpr double kMaxDrift2 = 1e-2;
constexpr int kMaxReplaceGap = 2;   // largest check interval with replacement
constexpr int kWidth = MFGP_MAX_D + 1;   // adjoint partial width

// ---------------------------------------------------------------- persistent kernels

__global__ void reset_counter_kernel(int* counter) {
    if (threadIdx.x == 0) *counter = 0;
}

// A problem is live while any of its t columns is active in CG (`live` holds
// the per-column active flags, problem b's at [b t, b t + t)).  The persistent
// sweeps skip the tiles of problems that are not (nothing of theirs is read
// afterwards: the CG update leaves inactive columns untouched); `live` is
// NULL outside CG (autotuner), where every tile runs.  The flags were written
// by the previous launch on the stream; the check is uniform over the
// workgroup (the tile index is), so no barrier is skipped by part of it.
__device__ __forceinline__ bool problem_live(const int* __restrict__ live, int b, int t) {
    if (!live) return true;
    int any = 0;
    for (int c = 0; c < t; ++c) any |= live[b * t + c];
    return any != 0;
}

template <int FAM, int TB>
__global__ __launch_bounds__(kBlock) void batch_sweep_kernel(
    const BTile* __restrict__ queue, int ntiles, int* counter, const BProb* __restrict__ probs,
    const float* __restrict__ U, const float* __restrict__ V, float* __restrict__ partial,
    const int* __restrict__ live) {
    __shared__ int s_k;
    for (;;) {
        if (threadIdx.x == 0) s_k = atomicAdd(counter, 1);
        __syncthreads();
        const int k = __builtin_amdgcn_readfirstlane(s_k);
        __syncthreads();
        if (k >= ntiles) break;
        const BTile tl = queue[k];
        if (!problem_live(live, tl.b, TB)) continue;
        const BProb pb = probs[tl.b];
        const int64_t i = static_cast<int64_t>(tl.rb) * kBlock + threadIdx.x;
        const int64_t ii = i < pb.n ? i : pb.n - 1;
        const int64_t j0 = static_cast<int64_t>(tl.ch) * pb.jchunk;
        const int64_t jend = j0 + pb.jchunk < pb.n ? j0 + pb.jchunk : pb.n;
        const int cnt = j0 < jend ? static_cast<int>(jend - j0) : 0;
        const float* Ub = U + pb.u_off;
        const float* Vb = V + pb.row_off * TB;
        float acc[TB];
        switch (pb.d) {
#define MFGP_BCASE(DV)                                                         \
    case DV: {                                                                 \
        float ui[DV];                                                          \
        _Pragma("unroll") for (int q = 0; q < DV; ++q) ui[q] = Ub[ii * DV + q]; \
        sweep_rows<FAM, DV, TB>(ui, Ub + j0 * DV, Vb + j0 * TB, cnt, acc);     \
    } break;
            MFGP_BCASE(1) MFGP_BCASE(2) MFGP_BCASE(3) MFGP_BCASE(4)
            MFGP_BCASE(5) MFGP_BCASE(6) MFGP_BCASE(7) MFGP_BCASE(8)
#undef MFGP_BCASE
            default:
#pragma unroll
                for (int c = 0; c < TB; ++c) acc[c] = 0.0f;
        }
        float* p = partial + (static_cast<int64_t>(tl.id) * kBlock + threadIdx.x) * TB;
#pragma unroll
        for (int c = 0; c < TB; ++c) p[c] = acc[c];
    }
}

template <int FAM, int TB>
__global__ __launch_bounds__(kBlock) void batch_adjoint_kernel(
    const BTile* __restrict__ queue, int ntiles, int* counter, const BProb* __restrict__ probs,
    const float* __restrict__ U, const float* __restrict__ A, const float* __restrict__ B, ColW w,
    double* __restrict__ partial) {
    __shared__ int s_k;
    __shared__ double red[kWidth * (kBlock / 64)];
    for (;;) {
        if (threadIdx.x == 0) s_k = atomicAdd(counter, 1);
        __syncthreads();
        const int k = __builtin_amdgcn_readfirstlane(s_k);
        __syncthreads();
        if (k >= ntiles) break;
        const BTile tl = queue[k];
        const BProb pb = probs[tl.b];
        const int64_t i = static_cast<int64_t>(tl.rb) * kBlock + threadIdx.x;
        const int64_t ii = i < pb.n ? i : pb.n - 1;
        const int64_t j0 = static_cast<int64_t>(tl.ch) * pb.jchunk;
        const int64_t jend = j0 + pb.jchunk < pb.n ? j0 + pb.jchunk : pb.n;
        const int cnt = j0 < jend ? static_cast<int>(jend - j0) : 0;
        const float* Ub = U + pb.u_off;
        const float* Ab = A + pb.row_off * TB;
        const float* Bb = B + pb.row_off * TB;
        float ai[TB];
#pragma unroll
        for (int c = 0; c < TB; ++c) ai[c] = i < pb.n ? Ab[ii * TB + c] * w.w[c] : 0.0f;
        double* out = partial + static_cast<int64_t>(tl.id) * kWidth;
        switch (pb.d) {
#define MFGP_ACASE(DV)                                                          \
    case DV: {                                                                  \
        float ui[DV];                                                           \
        _Pragma("unroll") for (int q = 0; q < DV; ++q) ui[q] = Ub[ii * DV + q];  \
        double v[DV + 1];                                                       \
        adjoint_rows<FAM, DV, TB>(ui, ai, Ub + j0 * DV, Bb + j0 * TB, cnt, v);  \
        block_sum_write<DV + 1>(v, red, out);                                   \
    } break;
            MFGP_ACASE(1) MFGP_ACASE(2) MFGP_ACASE(3) MFGP_ACASE(4)
            MFGP_ACASE(5) MFGP_ACASE(6) MFGP_ACASE(7) MFGP_ACASE(8)
#undef MFGP_ACASE
            default: break;
        }
        __syncthreads();   // red is reused by the next tile
    }
}

// Persistent batched sweep with the contraction on FP32 MFMA (t = 16 NT + TV):
// the same tile queue, each tile running the shared hybrid block body.
template <int FAM, int NT, int TV>
__global__ __launch_bounds__(kBlock) void batch_hyb_kernel(
    const BTile* __restrict__ queue, int ntiles, int* counter, const BProb* __restrict__ probs,
    const float* __restrict__ U, const float* __restrict__ F, int t, float* __restrict__ partial,
    const int* __restrict__ live) {
    __shared__ int s_k;
    for (;;) {
        if (threadIdx.x == 0) s_k = atomicAdd(counter, 1);
        __syncthreads();
        const int k = __builtin_amdgcn_readfirstlane(s_k);
        __syncthreads();
        if (k >= ntiles) break;
        const BTile tl = queue[k];
        if (!problem_live(live, tl.b, t)) continue;
        const BProb pb = probs[tl.b];
        const int64_t j0 = static_cast<int64_t>(tl.ch) * pb.jchunk;
        const float* Ub = U + pb.u_off;
        const float* Fb = F + pb.f_off;
        float* out = partial + static_cast<int64_t>(tl.id) * kBlock * t;
        const int64_t rbase = static_cast<int64_t>(tl.rb) * kBlock;
        switch (pb.d) {
#define MFGP_HCASE(DV) \
    case DV: hyb_block<FAM, DV, NT, TV>(Ub, Ub, Fb, pb.n, pb.n, t, rbase, j0, j0 + pb.jchunk, out); break;
            MFGP_HCASE(1) MFGP_HCASE(2) MFGP_HCASE(3) MFGP_HCASE(4)
            MFGP_HCASE(5) MFGP_HCASE(6) MFGP_HCASE(7) MFGP_HCASE(8)
#undef MFGP_HCASE
            default: break;
        }
    }
}

// Fragments of every problem's packed V block (layout as in the single-problem
// hybrid sweep), problem found by binary search over the fragment offsets.
// Fragments of V for the hybrid sweep, per problem (grid laid out per problem
// as in batch_reduce_kernel).  The fragments of a problem whose columns have
// all stopped are not read by the sweep, which skips its tiles: they are not
// packed either.
__global__ void batch_pack_hfrag_kernel(const float* __restrict__ V, const BProb* __restrict__ probs,
                                        const int* __restrict__ blk_prob, const int* __restrict__ blk_first,
                                        int t, int nt, int tv, float* __restrict__ F, const int* __restrict__ live) {
    const int b = blk_prob[blockIdx.x];
    if (!problem_live(live, b, t)) return;   // uniform over the block
    const BProb pb = probs[b];
    const unsigned W = static_cast<unsigned>(nt + tv);
    // a problem's fragments: ceil(n_b / 4) steps x 64 lanes x W < 2^32 (n_b <= 2^24)
    const unsigned cnt = static_cast<unsigned>((pb.n + kHK - 1) / kHK) * 64u * W;
    const unsigned loc = static_cast<unsigned>(blockIdx.x - blk_first[b]) * 256u + threadIdx.x;
    if (loc >= cnt) return;
    const int w = static_cast<int>(loc % W);
    const unsigned lq = loc / W;
    const int l = static_cast<int>(lq & 63u);
    const int64_t q = lq >> 6;
    const int64_t j = q * kHK + l / 16;
    const int c = w < nt ? tv + 16 * w + (l % 16) : w - nt;
    F[pb.f_off + loc] = (j < pb.n) ? V[(pb.row_off + j) * t + c] : 0.0f;
}

// Persistent batched sweep with the contraction on the bf16 matrix cores
// (the x1 / x2 / x3 forms of the single-problem BF16 sweep, same tile body).
template <int FAM, int NT, int SPLIT, int TV>
__global__ __launch_bounds__(kBlock) void batch_mfma_kernel(
    const BTile* __restrict__ queue, int ntiles, int* counter, const BProb* __restrict__ probs,
    const float* __restrict__ U, const bf16x8* __restrict__ Gh, const bf16x8* __restrict__ Gm,
    const bf16x8* __restrict__ Gl, const float* __restrict__ Gy, int t, float* __restrict__ partial,
    const int* __restrict__ live) {
    __shared__ int s_k;
    for (;;) {
        if (threadIdx.x == 0) s_k = atomicAdd(counter, 1);
        __syncthreads();
        const int k = __builtin_amdgcn_readfirstlane(s_k);
        __syncthreads();
        if (k >= ntiles) break;
        const BTile tl = queue[k];
        if (!problem_live(live, tl.b, t)) continue;
        const BProb pb = probs[tl.b];
        const int64_t j0 = static_cast<int64_t>(tl.ch) * pb.jchunk;   // multiple of 16
        const float* Ub = U + pb.u_off;
        float* out = partial + static_cast<int64_t>(tl.id) * kBlock * t;
        const int64_t rbase = static_cast<int64_t>(tl.rb) * kBlock;
        switch (pb.d) {
#define MFGP_GCASE(DV)                                                                                  \
    case DV:                                                                                            \
        mfma_block<FAM, DV, NT, SPLIT, TV>(Ub, Ub, Gh + pb.g_off, Gm + pb.g_off, Gl + pb.g_off,          \
                                           Gy + pb.y_off, pb.n, pb.n, t, rbase, j0, j0 + pb.jchunk, out); \
        break;
            MFGP_GCASE(1) MFGP_GCASE(2) MFGP_GCASE(3) MFGP_GCASE(4)
            MFGP_GCASE(5) MFGP_GCASE(6) MFGP_GCASE(7) MFGP_GCASE(8)
#undef MFGP_GCASE
            default: break;
        }
    }
}

// Largest b with offs[b] <= idx (offs ascending, offs[0] = 0).
__device__ __forceinline__ int find_slot(const int64_t* __restrict__ offs, int nprob, int64_t idx) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// BF16 fragments of every problem's packed V block (layout of the single-
// problem BF16 sweep) and, when tv, the FP32 copy of column 0.
__global__ void batch_pack_bfrag_kernel(const float* __restrict__ V, const BProb* __restrict__ probs,
                                        const int64_t* __restrict__ goffs, const int64_t* __restrict__ yoffs,
                                        int nprob, int t, int tv, int nt, int split, bf16x8* __restrict__ Gh,
                                        bf16x8* __restrict__ Gm, bf16x8* __restrict__ Gl,
                                        float* __restrict__ Gy, const int* __restrict__ live) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tv && idx < yoffs[nprob]) {
        const int b = find_slot(yoffs, nprob, idx);
        if (problem_live(live, b, t)) {
            const BProb pb = probs[b];
            const int64_t j = idx - pb.y_off;
            Gy[idx] = j < pb.n ? V[(pb.row_off + j) * t] : 0.0f;
        }
    }
    if (idx >= goffs[nprob]) return;
    const int bg = find_slot(goffs, nprob, idx);
    if (!problem_live(live, bg, t)) return;
    const BProb pb = probs[bg];
    const unsigned loc = static_cast<unsigned>(idx - pb.g_off);   // < 2^32 per problem
    const int l = static_cast<int>(loc & 63u);
    const unsigned f = loc >> 6;
    const int ct = static_cast<int>(f % static_cast<unsigned>(nt));
    const int64_t jt = f / static_cast<unsigned>(nt);
    bf16x8 h8, m8, l8;
    vfrag(V + pb.row_off * t, pb.n, t, tv, jt, ct, l, h8, m8, l8);
    Gh[idx] = h8;
    if (split >= 1) Gm[idx] = m8;
    if (split >= 2) Gl[idx] = l8;
}

// ---------------------------------------------------------------- batched reductions

// out[problem rows, c] = s2 sum over the row's tile partials + sigma2 V
// (columns not active in CG, live non-NULL, are not needed: skipped).  The
// grid is laid out per problem (blk_prob: problem of each 256-thread block,
// blk_first: the problem's first block), so the thread finds its problem and
// its element (i, c) of that problem with one table load and 32-bit index
// arithmetic (n_b t < 2^32).
__global__ void batch_reduce_kernel(const float* __restrict__ partial, const BProb* __restrict__ probs,
                                    const int* __restrict__ blk_prob, const int* __restrict__ blk_first,
                                    int t, const float* __restrict__ Vself, float* __restrict__ out,
                                    const int* __restrict__ live) {
    const int b = blk_prob[blockIdx.x];
    const BProb pb = probs[b];
    const unsigned loc = static_cast<unsigned>(blockIdx.x - blk_first[b]) * 256u + threadIdx.x;
    if (loc >= static_cast<unsigned>(pb.n) * static_cast<unsigned>(t)) return;
    const unsigned i = loc / static_cast<unsigned>(t);
    const int c = static_cast<int>(loc - i * static_cast<unsigned>(t));
    if (live && !live[b * t + c]) return;
    const int64_t rb = i / kBlock;
    const int64_t li = i % kBlock;
    double acc = 0.0;
    for (int ch = 0; ch < pb.chunks; ++ch) {
        const int64_t tile = pb.tile_base + rb * pb.chunks + ch;
        acc += static_cast<double>(partial[(tile * kBlock + li) * t + c]);
    }
    const int64_t idx = pb.row_off * t + loc;
    out[idx] = static_cast<float>(static_cast<double>(pb.s2) * acc +
                                  static_cast<double>(pb.sig2) * static_cast<double>(Vself[idx]));
}

// Segment k: rows [r0, r1) of one problem; striped over S = floor(256/t)*t threads.
template <typename TA, typename TB_>
__global__ __launch_bounds__(256) void bdot_stage1(const TA* __restrict__ a, const TB_* __restrict__ b,
                                                   const BSeg* __restrict__ segs, int t,
                                                   double* __restrict__ part) {
    __shared__ double lds[256];
    const BSeg sg = segs[blockIdx.x];
    const int S = (256 / t) * t;
    const int k = threadIdx.x;
    double acc = 0.0;
    if (k < S)
        for (int64_t e = sg.r0 * t + k; e < sg.r1 * t; e += S)
            acc = fma(static_cast<double>(a[e]), static_cast<double>(b[e]), acc);
    lds[k] = k < S ? acc : 0.0;
    __syncthreads();
    for (int c = threadIdx.x; c < t; c += 256) {
        double s = 0.0;
        for (int q = c; q < S; q += t) s += lds[q];
        part[static_cast<int64_t>(blockIdx.x) * t + c] = s;
    }
}

__global__ void bdot_stage2(const double* __restrict__ part, const int* __restrict__ seg_first,
                            int nprob, int t, double* __restrict__ out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nprob * t) return;
    const int b = idx / t;
    const int c = idx % t;
    double s = 0.0;
    for (int k = seg_first[b]; k < seg_first[b + 1]; ++k) s += part[static_cast<int64_t>(k) * t + c];
    out[idx] = s;
}

// x += alpha p, r -= alpha Ap per (problem, column), striped r^2 partials.
__global__ __launch_bounds__(256) void bcg_update_kernel(CgState st, const BSeg* __restrict__ segs, int t,
                                                         double* __restrict__ part) {
    __shared__ double lds[256];
    const BSeg sg = segs[blockIdx.x];
    const int S = (256 / t) * t;
    const int k = threadIdx.x;
    double acc = 0.0;
    if (k < S) {
        const int c = k % t;
        const double a = st.alpha[sg.b * t + c];
        const float af = static_cast<float>(a);
        for (int64_t e = sg.r0 * t + k; e < sg.r1 * t; e += S) {
            if (a != 0.0) {
                st.x[e] = fma(a, static_cast<double>(st.p[e]), st.x[e]);
                st.r[e] = fmaf(-af, st.ap[e], st.r[e]);
            }
            const float r = st.r[e];
            acc = fma(static_cast<double>(r), static_cast<double>(r), acc);
        }
    }
    lds[k] = k < S ? acc : 0.0;
    __syncthreads();
    for (int c = threadIdx.x; c < t; c += 256) {
        double s = 0.0;
        for (int q = c; q < S; q += t) s += lds[q];
        part[static_cast<int64_t>(blockIdx.x) * t + c] = s;
    }
}

// p = r + beta p for active (problem, column); restart: r = fl32(R64), p = r.
// p = r + beta p for the active columns: threads k < S = floor(256 / t) t
// stride the segment by S, so thread k always holds column k % t (no
// per-element division) and reads that column's flag and beta once.
__global__ __launch_bounds__(256) void bcg_p_kernel(CgState st, const BSeg* __restrict__ segs, int t) {
    const BSeg sg = segs[blockIdx.x];
    const int S = (256 / t) * t;
    const int k = threadIdx.x;
    if (k >= S) return;
    const int q = sg.b * t + k % t;
    if (!st.active[q]) return;
    const float beta = static_cast<float>(st.beta[q]);
    for (int64_t e = sg.r0 * t + k; e < sg.r1 * t; e += S) st.p[e] = fmaf(beta, st.p[e], st.r[e]);
}

__global__ __launch_bounds__(256) void bcg_restart_kernel(CgState st, const BSeg* __restrict__ segs, int t,
                                                          const double* __restrict__ R64,
                                                          const int* __restrict__ restart) {
    const BSeg sg = segs[blockIdx.x];
    for (int64_t e = sg.r0 * t + threadIdx.x; e < sg.r1 * t; e += 256) {
        if (restart[sg.b * t + static_cast<int>(e % t)]) {
            const float r = static_cast<float>(R64[e]);
            st.r[e] = r;
            st.p[e] = r;
        }
    }
}

// Residual replacement for flagged (problem, column), as in the single-problem
// solver: r = fl32(R64) and p += r_new - r_old (the direction re-formed from
// the replaced residual); only columns with small drift are flagged.
__global__ __launch_bounds__(256) void bcg_replace_kernel(CgState st, const BSeg* __restrict__ segs, int t,
                                                          const double* __restrict__ R64,
                                                          const int* __restrict__ flag) {
    const BSeg sg = segs[blockIdx.x];
    for (int64_t e = sg.r0 * t + threadIdx.x; e < sg.r1 * t; e += 256)
        if (flag[sg.b * t + static_cast<int>(e % t)]) {
            const float rn = static_cast<float>(R64[e]);
            st.p[e] += rn - st.r[e];
            st.r[e] = rn;
        }
}

__global__ void bcg_set_rr_kernel(CgState st, int T, const int* __restrict__ flag,
                                  const double* __restrict__ rr_new) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < T && flag[q]) st.rr[q] = rr_new[q];
}

__global__ void bcg_init_kernel(CgState st, int T, double tol2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T) return;
    const bool finite = isfinite(st.bnorm2[q]) && isfinite(st.rr[q]);
    st.active[q] = (finite && st.bnorm2[q] > 0.0 && st.rr[q] > tol2 * st.bnorm2[q]) ? 1 : 0;
    st.status[q] = finite ? MFGP_OK : MFGP_BREAKDOWN;
    st.iters[q] = 0;
    st.lanlen[q] = 0;
    st.alpha[q] = 0.0;
    st.beta[q] = 0.0;
}

__global__ void bcg_alpha_kernel(CgState st, int T) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T) return;
    double a = 0.0;
    if (st.active[q]) {
        const double pap = st.pap[q];
        if (!(pap > 0.0) || !isfinite(pap) || !isfinite(st.rr[q])) {
            st.status[q] = MFGP_BREAKDOWN;
            st.active[q] = 0;
        } else {
            a = st.rr[q] / pap;
        }
    }
    st.alpha[q] = a;
}

__global__ void bcg_beta_kernel(CgState st, int T, const double* __restrict__ rrn_all, double tol2,
                                const int* __restrict__ log_coeffs, int max_iter) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T) return;
    const double rrn = rrn_all[q];
    double b = 0.0;
    if (st.active[q]) {
        b = rrn / st.rr[q];
        if (log_coeffs[q] && st.lanlen[q] < max_iter) {
            double* cf = st.coeff + (static_cast<int64_t>(q) * max_iter + st.lanlen[q]) * 2;
            cf[0] = st.alpha[q];
            cf[1] = b;
            st.lanlen[q] += 1;
        }
        st.iters[q] += 1;
        st.rr[q] = rrn;
        if (!isfinite(rrn)) {
            st.status[q] = MFGP_BREAKDOWN;
            st.active[q] = 0;
        } else if (rrn <= tol2 * st.bnorm2[q] || st.iters[q] >= max_iter) {
            st.active[q] = 0;
        }
    }
    st.beta[q] = b;
}

// Re-activate restarted columns with their new residual norm; a restarted
// column no longer records Lanczos coefficients (the tridiagonal of the SLQ
// belongs to its first cycle).
__global__ void bcg_activate_kernel(CgState st, int T, const int* __restrict__ restart,
                                    const double* __restrict__ rr_new, int* __restrict__ log_coeffs) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T) return;
    if (restart[q]) {
        st.active[q] = rr_new[q] > 0.0 ? 1 : 0;
        st.rr[q] = rr_new[q];
        log_coeffs[q] = 0;
    }
}

__global__ void adjoint_stage2_kernel(const double* __restrict__ partial, const BProb* __restrict__ probs,
                                      int nprob, double* __restrict__ out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nprob * kWidth) return;
    const int b = idx / kWidth;
    const int k = idx % kWidth;
    const BProb pb = probs[b];
    double s = 0.0;
    if (k <= pb.d) {
        const int ntile = pb.rowblocks * pb.chunks;
        for (int q = 0; q < ntile; ++q) s += partial[static_cast<int64_t>(pb.tile_base + q) * kWidth + k];
    }
    out[idx] = s;
}

__global__ void batch_pack_yz_kernel(const float* __restrict__ y, const float* __restrict__ Z,
                                     int64_t rows, int p, float* __restrict__ out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int t = p + 1;
    if (idx >= rows * t) return;
    const int64_t r = idx / t;
    const int c = static_cast<int>(idx % t);
    out[idx] = c == 0 ? y[r] : Z[r * p + (c - 1)];
}

__global__ void batch_set_col0_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                      int64_t rows, int t) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < rows) dst[r * t] = static_cast<float>(src[r * t]);
}

static inline unsigned nblocks(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

}  // namespace mfgp

// ---------------------------------------------------------------- the plan

using namespace mfgp;

struct mfgp_batch_plan_s {
    int nprob = 0;
    int p = 0, t = 0;
    int family = 0;
    int max_iter = 0;
    int tune = 0;
    int use_graph = 1;
    std::vector<int64_t> n, row_off, x_off;
    std::vector<mfgp_kernel> kern;
    int64_t rows = 0;          // sum n_b
    int64_t xelems = 0;        // packed X elements
    int64_t max_n = 0;
    int64_t tile_j = 0;        // tuned (0 = not yet)
    double tuned_ms = 0.0;
    int64_t graph_launches = 0;
    std::vector<BSeg> segs;
    std::vector<int> seg_first;
    std::vector<int64_t> row_offs;   // prefix [nprob + 1]
    std::vector<int64_t> frag_off;   // prefix [nprob + 1] of the MFMA fragments (floats)
    int hyb_nt = 0, hyb_tv = 0;      // t = 16 nt + tv with an MFMA-contraction kernel
    bool hybrid = false;
    std::vector<int64_t> gfrag_off;  // prefix [nprob + 1] of the BF16 fragments (bf16x8)
    std::vector<int64_t> y_off;      // prefix [nprob + 1] of the FP32 column-0 copies
    // Per-problem grids of the element-wise kernels: the problem of each
    // 256-thread block and each problem's first block (fragment packing of
    // the hybrid sweep; the reduction over n_b t outputs).
    std::vector<int> pack_blk, pack_first, red_blk, red_first;
    int precision = MFGP_FP32;       // precision of the current call's products
    // Capture stream (default priority, non-blocking): the caller's stream may
    // be the legacy NULL stream, which cannot be captured; the graph recorded
    // here is then launched on the caller's stream.
    hipStream_t cap_stream = nullptr;
    ~mfgp_batch_plan_s() {
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace mfgp {

static const int64_t kTileCandidates[] = {4096, 8192, 16384, 32768, 65536};
static const int64_t kDefaultTile = 8192;
static const int64_t kMinTile = 4096;

static void build_tiles(const mfgp_batch_plan_s& P, int64_t J, std::vector<BProb>& probs,
                        std::vector<BTile>& queue) {
    probs.resize(P.nprob);
    int base = 0;
    for (int b = 0; b < P.nprob; ++b) {
        BProb& pb = probs[b];
        const Operator op = make_operator(P.kern[b], nullptr, P.n[b], nullptr);
        pb.n = P.n[b];
        pb.row_off = P.row_off[b];
        pb.u_off = P.x_off[b];
        pb.d = P.kern[b].d;
        pb.rowblocks = static_cast<int>((pb.n + kBlock - 1) / kBlock);
        pb.chunks = static_cast<int>((pb.n + J - 1) / J);
        // whole MFMA steps of every form (4 j for FP32, 16 j for bf16)
        pb.jchunk = ((pb.n + pb.chunks - 1) / pb.chunks + kJT - 1) / kJT * kJT;
        pb.tile_base = base;
        pb.f_off = P.frag_off[b];
        pb.g_off = P.gfrag_off[b];
        pb.y_off = P.y_off[b];
        pb.s2 = op.s2;
        pb.sig2 = op.sig2;
        base += pb.rowblocks * pb.chunks;
    }
    queue.clear();
    queue.reserve(base);
    for (int b = 0; b < P.nprob; ++b) {
        const BProb& pb = probs[b];
        for (int rb = 0; rb < pb.rowblocks; ++rb)
            for (int ch = 0; ch < pb.chunks; ++ch)
                queue.push_back(BTile{b, rb, ch, pb.tile_base + rb * pb.chunks + ch});
    }
    // Longest processing time first: work of a tile = rows x j-range x d-ish cost.
    auto work = [&](const BTile& tl) {
        const BProb& pb = probs[tl.b];
        const int64_t rows = std::min<int64_t>(kBlock, pb.n - static_cast<int64_t>(tl.rb) * kBlock);
        const int64_t j0 = tl.ch * pb.jchunk;
        const int64_t js = std::min<int64_t>(pb.jchunk, pb.n - j0);
        return static_cast<double>(rows) * static_cast<double>(js) * (2.0 * pb.d + 4.0);
    };
    std::stable_sort(queue.begin(), queue.end(),
                     [&](const BTile& a, const BTile& b) { return work(a) > work(b); });
}

static int64_t max_tiles(const mfgp_batch_plan_s& P) {
    int64_t total = 0;
    for (int b = 0; b < P.nprob; ++b) {
        const int64_t rbk = (P.n[b] + kBlock - 1) / kBlock;
        const int64_t ch = (P.n[b] + kMinTile - 1) / kMinTile;
        total += rbk * ch;
    }
    return total;
}

struct BatchWs {
    float* U; float* Bm; double* X64; float* Zgen; double* coeff; float* R; float* P; float* AP;
    double* R64; double* scal; int* ints; double* dpart; double* tmp; double* resid; char* part;
    BTile* queue; BProb* probs; BSeg* segs; int* seg_first; int* counter;
    int* logflag;
    int* pack_blk; int* pack_first; int* red_blk; int* red_first;   // per-problem grids (plan)
    float* frag;      // MFMA fragments of the product's right-hand sides
    bf16x8* gh; bf16x8* gm; bf16x8* gl;   // BF16 fragments (three split pieces)
    float* gy;        // FP32 column 0 of the BF16 products
    int64_t* goffs;   // [nprob + 1] BF16 fragment offsets
    int64_t* yoffs;   // [nprob + 1] column-0 offsets
    int cus;          // compute units of the device (host value)
};

static BatchWs carve_batch(Carver& cv, const mfgp_batch_plan_s& P) {
    BatchWs w;
    w.cus = 256;
    const size_t rt = static_cast<size_t>(P.rows) * P.t;
    const size_t T = static_cast<size_t>(P.nprob) * P.t;
    const int64_t nt = max_tiles(P);
    w.U = cv.take<float>(P.xelems);
    w.Bm = cv.take<float>(rt);
    w.X64 = cv.take<double>(rt);
    w.Zgen = cv.take<float>(static_cast<size_t>(P.rows) * P.p);
    w.coeff = cv.take<double>(T * P.max_iter * 2);
    w.R = cv.take<float>(rt);
    w.P = cv.take<float>(rt);
    w.AP = cv.take<float>(rt);
    w.R64 = cv.take<double>(rt);
    w.scal = cv.take<double>(8 * T);
    w.ints = cv.take<int>(6 * T);
    w.dpart = cv.take<double>(P.segs.size() * P.t + 64);
    w.tmp = cv.take<double>(4 * T + 64);
    size_t resid = 0;
    for (int b = 0; b < P.nprob; ++b) resid = std::max(resid, resid_scratch_doubles(P.n[b], P.t));
    w.resid = cv.take<double>(resid);
    const size_t part_sweep = static_cast<size_t>(nt) * kBlock * P.t * sizeof(float);
    const size_t part_adj = static_cast<size_t>(nt) * kWidth * sizeof(double) + (P.nprob * kWidth + 64) * sizeof(double);
    w.part = cv.take<char>(std::max(part_sweep, part_adj));
    w.queue = cv.take<BTile>(nt);
    w.probs = cv.take<BProb>(P.nprob);
    w.segs = cv.take<BSeg>(P.segs.size());
    w.seg_first = cv.take<int>(P.nprob + 1);
    w.counter = cv.take<int>(64);
    w.logflag = cv.take<int>(T + 64);   // per column: records Lanczos coefficients
    w.pack_blk = cv.take<int>(P.pack_blk.size());
    w.pack_first = cv.take<int>(P.pack_first.size());
    w.red_blk = cv.take<int>(P.red_blk.size());
    w.red_first = cv.take<int>(P.red_first.size());
    w.frag = cv.take<float>(P.frag_off.empty() ? 0 : P.frag_off.back());
    const size_t g = P.gfrag_off.empty() ? 0 : static_cast<size_t>(P.gfrag_off.back());
    w.gh = cv.take<bf16x8>(g);
    w.gm = cv.take<bf16x8>(g);
    w.gl = cv.take<bf16x8>(g);
    w.gy = cv.take<float>(P.y_off.empty() ? 0 : static_cast<size_t>(P.y_off.back()));
    w.goffs = cv.take<int64_t>(P.nprob + 1);
    w.yoffs = cv.take<int64_t>(P.nprob + 1);
    return w;
}

// Resident workgroups of the persistent kernels: 8 per CU (the CU count is
// read by the caller before any graph capture begins).
static int persistent_grid(int ntiles, int cus) {
    return static_cast<int>(std::min<int64_t>(ntiles, static_cast<int64_t>(cus) * 8));
}

template <int FAM>
static hipError_t launch_bsweep_f(int tb, const BatchWs& w, int ntiles, const float* V, float* part,
                                  const int* live, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(persistent_grid(ntiles, w.cus));
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, w.counter);
    switch (tb) {
#define MFGP_C(TBV)                                                                                 \
    case TBV:                                                                                       \
        hipLaunchKernelGGL((batch_sweep_kernel<FAM, TBV>), dim3(grid), dim3(kBlock), 0, s, w.queue, \
                           ntiles, w.counter, w.probs, w.U, V, part, live);                        \
        return hipGetLastError();
        MFGP_TB_LIST(MFGP_C)
#undef MFGP_C
        default: return hipErrorInvalidValue;
    }
}

template <int FAM>
static hipError_t launch_bhyb_f(const mfgp_batch_plan_s& P, const BatchWs& w, int ntiles, float* part,
                                const int* live, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(persistent_grid(ntiles, w.cus));
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, w.counter);
#define MFGP_HB(NTV, TVV)                                                                           \
    if (P.hyb_nt == NTV && P.hyb_tv == TVV) {                                                       \
        hipLaunchKernelGGL((batch_hyb_kernel<FAM, NTV, TVV>), dim3(grid), dim3(kBlock), 0, s, w.queue, \
                           ntiles, w.counter, w.probs, w.U, w.frag, P.t, part, live);               \
        return hipGetLastError();                                                                   \
    }
    MFGP_HB(1, 0) MFGP_HB(1, 1) MFGP_HB(2, 0) MFGP_HB(2, 1)
#undef MFGP_HB
    return hipErrorInvalidValue;
}

// Pack the fragments of V for all problems, then run the persistent hybrid sweep.
static hipError_t launch_bhyb(const mfgp_batch_plan_s& P, const BatchWs& w, int ntiles, const float* V,
                              float* part, const int* live, hipStream_t s) {
    hipLaunchKernelGGL(batch_pack_hfrag_kernel, dim3(static_cast<unsigned>(P.pack_blk.size())), dim3(256), 0,
                       s, V, w.probs, w.pack_blk, w.pack_first, P.t, P.hyb_nt, P.hyb_tv, w.frag, live);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (P.family) {
        case MFGP_RBF: return launch_bhyb_f<MFGP_RBF>(P, w, ntiles, part, live, s);
        case MFGP_MATERN12: return launch_bhyb_f<MFGP_MATERN12>(P, w, ntiles, part, live, s);
        case MFGP_MATERN32: return launch_bhyb_f<MFGP_MATERN32>(P, w, ntiles, part, live, s);
        default: return launch_bhyb_f<MFGP_MATERN52>(P, w, ntiles, part, live, s);
    }
}

static hipError_t launch_bsweep(int family, int tb, const BatchWs& w, int ntiles, const float* V,
                                float* part, const int* live, hipStream_t s) {
    switch (family) {
        case MFGP_RBF: return launch_bsweep_f<MFGP_RBF>(tb, w, ntiles, V, part, live, s);
        case MFGP_MATERN12: return launch_bsweep_f<MFGP_MATERN12>(tb, w, ntiles, V, part, live, s);
        case MFGP_MATERN32: return launch_bsweep_f<MFGP_MATERN32>(tb, w, ntiles, V, part, live, s);
        default: return launch_bsweep_f<MFGP_MATERN52>(tb, w, ntiles, V, part, live, s);
    }
}

template <int FAM>
static hipError_t launch_badj_f(int tb, const BatchWs& w, int ntiles, const float* A, const float* B,
                                const ColW& cw, double* part, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(persistent_grid(ntiles, w.cus));
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, w.counter);
    switch (tb) {
#define MFGP_C(TBV)                                                                                   \
    case TBV:                                                                                         \
        hipLaunchKernelGGL((batch_adjoint_kernel<FAM, TBV>), dim3(grid), dim3(kBlock), 0, s, w.queue, \
                           ntiles, w.counter, w.probs, w.U, A, B, cw, part);                         \
        return hipGetLastError();
        MFGP_TB_LIST(MFGP_C)
#undef MFGP_C
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_badj(int family, int tb, const BatchWs& w, int ntiles, const float* A,
                              const float* B, const ColW& cw, double* part, hipStream_t s) {
    switch (family) {
        case MFGP_RBF: return launch_badj_f<MFGP_RBF>(tb, w, ntiles, A, B, cw, part, s);
        case MFGP_MATERN12: return launch_badj_f<MFGP_MATERN12>(tb, w, ntiles, A, B, cw, part, s);
        case MFGP_MATERN32: return launch_badj_f<MFGP_MATERN32>(tb, w, ntiles, A, B, cw, part, s);
        default: return launch_badj_f<MFGP_MATERN52>(tb, w, ntiles, A, B, cw, part, s);
    }
}

// One batched product AP = K_y P (persistent sweep + fixed-order reduce), timed.
template <int FAM>
static hipError_t launch_bmfma_f(const mfgp_batch_plan_s& P, const BatchWs& w, int ntiles, int nt, int split,
                                 int tv, float* part, const int* live, hipStream_t s) {
    const unsigned grid = static_cast<unsigned>(persistent_grid(ntiles, w.cus));
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, w.counter);
#define MFGP_GB(NTV, SPV, TVV)                                                                        \
    if (nt == NTV && split == SPV && tv == TVV) {                                                     \
        hipLaunchKernelGGL((batch_mfma_kernel<FAM, NTV, SPV, TVV>), dim3(grid), dim3(kBlock), 0, s,   \
                           w.queue, ntiles, w.counter, w.probs, w.U, w.gh, w.gm, w.gl, w.gy, P.t, part, \
                           live);                                                                     \
        return hipGetLastError();                                                                     \
    }
    MFGP_GB(1, 0, 0) MFGP_GB(1, 1, 0) MFGP_GB(1, 2, 0) MFGP_GB(1, 0, 1) MFGP_GB(1, 1, 1) MFGP_GB(1, 2, 1)
#undef MFGP_GB
    return hipErrorInvalidValue;
}

// Pack the BF16 fragments of all problems, then run the persistent BF16 sweep.
static hipError_t launch_bmfma(const mfgp_batch_plan_s& P, const BatchWs& w, int ntiles, const float* V,
                               float* part, const int* live, hipStream_t s) {
    const int tv = vec_cols(P.t), nt = col_tiles(P.t), split = split_of(P.precision);
    const int64_t total = std::max<int64_t>(P.gfrag_off.back(), P.y_off.back());
    hipLaunchKernelGGL(batch_pack_bfrag_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0,
                       s, V, w.probs, w.goffs, w.yoffs, P.nprob, P.t, tv, nt, split, w.gh, w.gm, w.gl, w.gy,
                       live);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (P.family) {
        case MFGP_RBF: return launch_bmfma_f<MFGP_RBF>(P, w, ntiles, nt, split, tv, part, live, s);
        case MFGP_MATERN12: return launch_bmfma_f<MFGP_MATERN12>(P, w, ntiles, nt, split, tv, part, live, s);
        case MFGP_MATERN32: return launch_bmfma_f<MFGP_MATERN32>(P, w, ntiles, nt, split, tv, part, live, s);
        default: return launch_bmfma_f<MFGP_MATERN52>(P, w, ntiles, nt, split, tv, part, live, s);
    }
}

static bool is_bf16(int precision) {
    return precision == MFGP_BF16X1 || precision == MFGP_BF16X2 || precision == MFGP_BF16X3;
}

// One batched entry sweep in the precision of the current call.
// live: the CG active flags (tiles of finished problems are skipped), or NULL.
static hipError_t launch_batched_sweep(const mfgp_batch_plan_s& P, const BatchWs& w, int ntiles,
                                       const float* V, float* part, const int* live, hipStream_t s) {
    if (is_bf16(P.precision)) return launch_bmfma(P, w, ntiles, V, part, live, s);
    if (P.hybrid && (P.precision == MFGP_FP32 || P.precision == MFGP_FP32_DIRECT))
        return launch_bhyb(P, w, ntiles, V, part, live, s);
    return launch_bsweep(P.family, P.t, w, ntiles, V, part, live, s);
}

static hipError_t batch_apply(const mfgp_batch_plan_s& P, const BatchWs& w, int ntiles,
                              const float* V, float* out, const int* live, hipStream_t s) {
    void* tok = timing_begin(s);
    hipError_t e = launch_batched_sweep(P, w, ntiles, V, reinterpret_cast<float*>(w.part), live, s);
    if (e != hipSuccess) return e;
    double ent = 0.0, fl = 0.0;
    if (timing_on())
        for (int b = 0; b < P.nprob; ++b) {
            const double e2 = static_cast<double>(P.n[b]) * static_cast<double>(P.n[b]);
            ent += e2;
            fl += e2 * sweep_flops_per_entry(P.family, P.kern[b].d, P.t, false);
        }
    timing_end(tok, s, is_bf16(P.precision) ? kSweepMfma : kSweepF32, ent, fl);
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(static_cast<unsigned>(P.red_blk.size())), dim3(256), 0, s,
                       reinterpret_cast<const float*>(w.part), w.probs, w.red_blk, w.red_first, P.t, V, out,
                       live);
    return hipGetLastError();
}

static hipError_t bdots_ff(const mfgp_batch_plan_s& P, const BatchWs& w, const float* a, const float* b,
                           double* out, hipStream_t s) {
    hipLaunchKernelGGL((bdot_stage1<float, float>), dim3(static_cast<unsigned>(P.segs.size())), dim3(256),
                       0, s, a, b, w.segs, P.t, w.dpart);
    hipLaunchKernelGGL(bdot_stage2, dim3(nblocks(static_cast<int64_t>(P.nprob) * P.t)), dim3(256), 0, s,
                       w.dpart, w.seg_first, P.nprob, P.t, out);
    return hipGetLastError();
}
static hipError_t bdots_dd(const mfgp_batch_plan_s& P, const BatchWs& w, const double* a,
                           const double* b, double* out, hipStream_t s) {
    hipLaunchKernelGGL((bdot_stage1<double, double>), dim3(static_cast<unsigned>(P.segs.size())), dim3(256),
                       0, s, a, b, w.segs, P.t, w.dpart);
    hipLaunchKernelGGL(bdot_stage2, dim3(nblocks(static_cast<int64_t>(P.nprob) * P.t)), dim3(256), 0, s,
                       w.dpart, w.seg_first, P.nprob, P.t, out);
    return hipGetLastError();
}
static hipError_t bdots_df(const mfgp_batch_plan_s& P, const BatchWs& w, const double* a,
                           const float* b, double* out, hipStream_t s) {
    hipLaunchKernelGGL((bdot_stage1<double, float>), dim3(static_cast<unsigned>(P.segs.size())), dim3(256),
                       0, s, a, b, w.segs, P.t, w.dpart);
    hipLaunchKernelGGL(bdot_stage2, dim3(nblocks(static_cast<int64_t>(P.nprob) * P.t)), dim3(256), 0, s,
                       w.dpart, w.seg_first, P.nprob, P.t, out);
    return hipGetLastError();
}

// One CG iteration for the whole batch (all launches on s; capturable).
static hipError_t batch_iteration(const mfgp_batch_plan_s& P, const BatchWs& w, const CgState& st,
                                  int ntiles, double tol, hipStream_t s) {
    const int T = P.nprob * P.t;
    hipError_t e = batch_apply(P, w, ntiles, st.p, st.ap, st.active, s);
    if (e != hipSuccess) return e;
    e = bdots_ff(P, w, st.p, st.ap, st.pap, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bcg_alpha_kernel, dim3(nblocks(T)), dim3(256), 0, s, st, T);
    hipLaunchKernelGGL(bcg_update_kernel, dim3(static_cast<unsigned>(P.segs.size())), dim3(256), 0, s, st,
                       w.segs, P.t, w.dpart);
    double* rrn = w.tmp + 3 * T;
    hipLaunchKernelGGL(bdot_stage2, dim3(nblocks(T)), dim3(256), 0, s, w.dpart, w.seg_first, P.nprob, P.t, rrn);
    hipLaunchKernelGGL(bcg_beta_kernel, dim3(nblocks(T)), dim3(256), 0, s, st, T, rrn, tol * tol,
                       w.logflag, P.max_iter);
    hipLaunchKernelGGL(bcg_p_kernel, dim3(static_cast<unsigned>(P.segs.size())), dim3(256), 0, s, st,
                       w.segs, P.t);
    return hipGetLastError();
}

#define B_CHECK(expr)                          \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) {                \
            set_last_hip_error(e_);            \
            return MFGP_ERR_HIP;               \
        }                                      \
    } while (0)

static int upload_tiles(const mfgp_batch_plan_s& P, const BatchWs& w, int64_t J, int& ntiles,
                        std::vector<BProb>& probs, std::vector<BTile>& queue, hipStream_t s) {
    build_tiles(P, J, probs, queue);
    ntiles = static_cast<int>(queue.size());
    B_CHECK(hipMemcpyAsync(w.probs, probs.data(), probs.size() * sizeof(BProb), hipMemcpyHostToDevice, s));
    B_CHECK(hipMemcpyAsync(w.queue, queue.data(), queue.size() * sizeof(BTile), hipMemcpyHostToDevice, s));
    const std::vector<int>* maps[4] = {&P.pack_blk, &P.pack_first, &P.red_blk, &P.red_first};
    int* dst[4] = {w.pack_blk, w.pack_first, w.red_blk, w.red_first};
    for (int k = 0; k < 4; ++k)
        if (!maps[k]->empty())
            B_CHECK(hipMemcpyAsync(dst[k], maps[k]->data(), maps[k]->size() * sizeof(int), hipMemcpyHostToDevice, s));
    B_CHECK(hipStreamSynchronize(s));
    return MFGP_OK;
}

// Autotuner: time one batched sweep per candidate tile length on this batch
// and keep the fastest (ties to the longer tile).
static int tune_tiles(mfgp_batch_plan_s& P, const BatchWs& w, const float* V, hipStream_t s) {
    hipEvent_t a, b;
    B_CHECK(hipEventCreate(&a));
    B_CHECK(hipEventCreate(&b));
    double best = 1e300;
    int64_t bestJ = kDefaultTile;
    std::vector<BProb> probs;
    std::vector<BTile> queue;
    for (int64_t J : kTileCandidates) {
        int ntiles = 0;
        int st = upload_tiles(P, w, J, ntiles, probs, queue, s);
        if (st != MFGP_OK) return st;
        auto sweep = [&]() {
            return launch_batched_sweep(P, w, ntiles, V, reinterpret_cast<float*>(w.part), nullptr, s);
        };
        B_CHECK(sweep());  // warm
        B_CHECK(hipEventRecord(a, s));
        for (int r = 0; r < 2; ++r) B_CHECK(sweep());
        B_CHECK(hipEventRecord(b, s));
        B_CHECK(hipEventSynchronize(b));
        float ms = 0.0f;
        B_CHECK(hipEventElapsedTime(&ms, a, b));
        if (ms * 0.5 < best * 0.98) {
            best = ms * 0.5;
            bestJ = J;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    P.tile_j = bestJ;
    P.tuned_ms = best;
    return MFGP_OK;
}

static double lengthscale_factor_b(int family, double l) {
    const double c = family_scale(family);
    switch (family) {
        case MFGP_RBF: return 1.0 / (c * c * l);
        case MFGP_MATERN12: return 1.0 / (c * l);
        case MFGP_MATERN32: return 3.0 / (c * c * l);
        default: return (5.0 / 3.0) / (c * c * l);
    }
}

}  // namespace mfgp

// Stochastic Lanczos quadratures (Sec. 3 "Inference") of the batch's probe
// columns on host threads.  A problem's Lanczos coefficients are recorded in
// its columns' first cycles only and never change once every column of the
// problem has stopped for good, so its quadratures are queued then and run
// while the other problems keep iterating; the last problems' are queued when
// the solve ends.  Each column is computed by one thread into its own slots
// (qv[q], qs[q]); the owner joins the threads before reading them, also on an
// error return (the destructor drops what is still queued).
namespace {
struct SlqQueue {
    std::vector<std::vector<double>> cf;   // [T] coefficients (alpha, beta) of column q
    std::vector<int> len;                  // [T] their count
    std::vector<double> zn;                // [T] ||z_q||^2
    std::vector<double> qv;                // [T] quadrature of column q
    std::vector<int> qs;                   // [T] its status
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int> todo;
    bool closing = false, dropping = false;
    std::vector<std::thread> pool;

    explicit SlqQueue(int T) : cf(T), len(T, 0), zn(T, 0.0), qv(T, 0.0), qs(T, MFGP_OK) {}
    void run(int q) { qs[q] = len[q] < 1 ? MFGP_BREAKDOWN : mfgp_slq_quadrature(cf[q].data(), len[q], zn[q], &qv[q]); }
    // as many threads as the system gives, up to nth (none: finish() runs
    // the queue on the calling thread)
    void start(int nth) {
        for (int k = 0; k < nth; ++k) {
            try {
                pool.emplace_back([this]() {
                    for (;;) {
                        int q;
                        {
                            std::unique_lock<std::mutex> lk(mu);
                            cv.wait(lk, [this]() { return closing || !todo.empty(); });
                            if (todo.empty() || dropping) return;
                            q = todo.front();
                            todo.pop_front();
                        }
                        run(q);
                    }
                });
            } catch (...) {
                break;
            }
        }
    }
    void push(int q) {
        {
            std::lock_guard<std::mutex> lk(mu);
            todo.push_back(q);
        }
        cv.notify_one();
    }
    // wait for every queued column (drop == false) or for the running ones only
    void finish(bool drop) {
        {
            std::lock_guard<std::mutex> lk(mu);
            closing = true;
            dropping = drop;
        }
        cv.notify_all();
        for (auto& th : pool)
            if (th.joinable()) th.join();
        pool.clear();
        if (!drop)   // what no thread took (none could be started)
            for (; !todo.empty(); todo.pop_front()) run(todo.front());
        todo.clear();
    }
    ~SlqQueue() { finish(true); }
};
}  // namespace

extern "C" {

int mfgp_batch_plan_create(const mfgp_batch* batch, int32_t num_probes, int32_t max_iter, int32_t tune,
                           int32_t use_graph, mfgp_batch_plan* plan) {
    if (!batch || !plan || batch->nprob < 1 || !batch->n || !batch->row_off || !batch->x_off || !batch->kern)
        return MFGP_ERR_ARG;
    if (num_probes < 1 || max_iter < 0) return MFGP_ERR_ARG;
    const int t = num_probes + 1;
    bool tb_ok = false;
#define MFGP_T(TBV) tb_ok = tb_ok || (t == TBV);
    MFGP_TB_LIST(MFGP_T)
#undef MFGP_T
    if (!tb_ok) return MFGP_UNSUPPORTED;
    const int fam = batch->kern[0].family;
    if (fam == MFGP_PERIODIC || fam == MFGP_LINEAR) return MFGP_UNSUPPORTED;
    if (fam < MFGP_RBF || fam > MFGP_MATERN52) return MFGP_ERR_ARG;
    auto* P = new (std::nothrow) mfgp_batch_plan_s();
    if (!P) {
        set_last_hip_error(hipErrorOutOfMemory);
        return MFGP_ERR_HIP;
    }
    P->nprob = batch->nprob;
    P->p = num_probes;
    P->t = t;
    P->family = fam;
    P->tune = tune;
    P->use_graph = use_graph;
    int64_t maxn = 0;
    for (int b = 0; b < batch->nprob; ++b) {
        const mfgp_kernel& k = batch->kern[b];
        const int64_t n = batch->n[b];
        if (k.next || k.times) {
            delete P;
            return MFGP_UNSUPPORTED;   // kernel sums and products are not batched
        }
        bool ok = n >= 1 && k.family == fam && k.d >= 1 && k.d <= MFGP_MAX_D && std::isfinite(k.outputscale) &&
                  k.outputscale > 0.0f && std::isfinite(k.noise) && k.noise > 0.0f &&
                  batch->row_off[b] >= 0 && batch->x_off[b] >= 0;
        const int nl = k.ard ? k.d : 1;
        for (int q = 0; q < nl && ok; ++q) ok = std::isfinite(k.lengthscale[q]) && k.lengthscale[q] > 0.0f;
        if (!ok) {
            delete P;
            return MFGP_ERR_ARG;
        }
        if (n > (int64_t(1) << 24)) {   // per-problem fragment indices are 32-bit
            delete P;
            return MFGP_UNSUPPORTED;
        }
        P->n.push_back(n);
        P->row_off.push_back(batch->row_off[b]);
        P->x_off.push_back(batch->x_off[b]);
        P->kern.push_back(k);
        P->rows = std::max<int64_t>(P->rows, batch->row_off[b] + n);
        P->xelems = std::max<int64_t>(P->xelems, batch->x_off[b] + n * k.d);
        maxn = std::max(maxn, n);
    }
    P->max_n = maxn;
    P->max_iter = max_iter > 0 ? max_iter
                               : static_cast<int>(std::min<int64_t>(std::max<int64_t>(2 * maxn, 64), 20000));
    // segments of <= kSegRows rows within one problem, and row-offset prefix
    P->seg_first.push_back(0);
    for (int b = 0; b < P->nprob; ++b) {
        for (int64_t r = 0; r < P->n[b]; r += kSegRows) {
            BSeg sg;
            sg.b = b;
            sg.pad = 0;
            sg.r0 = P->row_off[b] + r;
            sg.r1 = P->row_off[b] + std::min<int64_t>(P->n[b], r + kSegRows);
            P->segs.push_back(sg);
        }
        P->seg_first.push_back(static_cast<int>(P->segs.size()));
    }
    // rows are packed back to back in problem order (row_off[b] = sum of earlier n)
    int64_t acc_rows = 0;
    for (int b = 0; b < P->nprob; ++b) {
        if (P->row_off[b] != acc_rows) {
            delete P;
            return MFGP_ERR_ARG;
        }
        P->row_offs.push_back(acc_rows);
        acc_rows += P->n[b];
    }
    P->row_offs.push_back(acc_rows);
    P->hybrid = hybrid_supported(t);
    P->hyb_nt = t / 16;
    P->hyb_tv = t % 16;
    int64_t facc = 0;
    for (int b = 0; b < P->nprob; ++b) {
        P->frag_off.push_back(facc);
        if (P->hybrid) facc += (P->n[b] + kHK - 1) / kHK * 64 * (P->hyb_nt + P->hyb_tv);
    }
    P->frag_off.push_back(facc);
    // per-problem grids of 256-thread blocks
    auto block_map = [&](auto count, std::vector<int>& blk, std::vector<int>& first) {
        for (int b = 0; b < P->nprob; ++b) {
            first.push_back(static_cast<int>(blk.size()));
            const int64_t nb = (count(b) + 255) / 256;
            for (int64_t k = 0; k < nb; ++k) blk.push_back(b);
        }
        first.push_back(static_cast<int>(blk.size()));
    };
    if (P->hybrid)
        block_map([&](int b) { return P->frag_off[b + 1] - P->frag_off[b]; }, P->pack_blk, P->pack_first);
    block_map([&](int b) { return P->n[b] * t; }, P->red_blk, P->red_first);
    int64_t gacc = 0, yacc = 0;
    for (int b = 0; b < P->nprob; ++b) {
        const int64_t njt = (P->n[b] + kJT - 1) / kJT;
        P->gfrag_off.push_back(gacc);
        P->y_off.push_back(yacc);
        gacc += njt * col_tiles(t) * 64;
        yacc += njt * kJT;
    }
    P->gfrag_off.push_back(gacc);
    P->y_off.push_back(yacc);
    *plan = P;
    return MFGP_OK;
}

int mfgp_batch_plan_destroy(mfgp_batch_plan plan) {
    delete plan;
    return MFGP_OK;
}

size_t mfgp_batch_workspace_bytes(mfgp_batch_plan plan) {
    if (!plan) return 0;
    Carver cv(nullptr);
    carve_batch(cv, *plan);
    return cv.off + 256;
}

int mfgp_batch_plan_info(mfgp_batch_plan plan, int64_t* tile_j, double* tuned_sweep_ms,
                         int64_t* graph_launches) {
    if (!plan) return MFGP_ERR_ARG;
    if (tile_j) *tile_j = plan->tile_j;
    if (tuned_sweep_ms) *tuned_sweep_ms = plan->tuned_ms;
    if (graph_launches) *graph_launches = plan->graph_launches;
    return MFGP_OK;
}

int mfgp_batch_mll_and_grad(mfgp_batch_plan plan, const float* X, const float* y, const float* Z,
                            const mfgp_cg_opts* opts, double* mll, double* logdet, double* grad,
                            mfgp_cg_info* info, void* ws, size_t ws_bytes, void* stream) {
    if (!plan || !X || !y || !opts || !mll || !ws) return MFGP_ERR_ARG;
    if (!std::isfinite(opts->tol) || !(opts->tol > 0.0) || opts->max_iter < 0) return MFGP_ERR_ARG;
    if (opts->precision < MFGP_FP32 || opts->precision > MFGP_FP32_GRAM) return MFGP_ERR_ARG;
    if (opts->precision == MFGP_FP32_GRAM) return MFGP_UNSUPPORTED;   // batched sweeps: direct differences
    if (is_bf16(opts->precision) && col_tiles(plan->t) != 1) return MFGP_UNSUPPORTED;
    if (ws_bytes < mfgp_batch_workspace_bytes(plan)) return MFGP_ERR_WORKSPACE;
    mfgp_batch_plan_s& P = *plan;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    BatchWs w = carve_batch(cv, P);
    {
        int dev = 0;
        w.cus = 256;
        B_CHECK(hipGetDevice(&dev));
        B_CHECK(hipDeviceGetAttribute(&w.cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    const int t = P.t, p = P.p, nprob = P.nprob;
    const int T = nprob * t;
    const int64_t rt = P.rows * t;
    const double tol = opts->tol;
    const int max_iter = P.max_iter;
    const int max_refine = opts->max_refine >= 0 ? opts->max_refine : 8;

    // Static descriptors and prescaled coordinates.
    B_CHECK(hipMemcpyAsync(w.segs, P.segs.data(), P.segs.size() * sizeof(BSeg), hipMemcpyHostToDevice, s));
    B_CHECK(hipMemcpyAsync(w.seg_first, P.seg_first.data(), P.seg_first.size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
    B_CHECK(hipMemcpyAsync(w.goffs, P.gfrag_off.data(), P.gfrag_off.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    B_CHECK(hipMemcpyAsync(w.yoffs, P.y_off.data(), P.y_off.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    if (P.precision != opts->precision) {
        P.precision = opts->precision;
        P.tile_j = 0;   // tile lengths are tuned per precision
    }
    std::vector<Operator> ops(nprob);
    for (int b = 0; b < nprob; ++b) {
        ops[b] = make_operator(P.kern[b], X + P.x_off[b], P.n[b], w.U + P.x_off[b]);
        B_CHECK(prescale(ops[b], s));
    }
    const float* Zp = Z;
    if (!Zp) {
        for (int b = 0; b < nprob; ++b)
            B_CHECK(launch_rademacher(opts->probe_seed + static_cast<uint64_t>(b), P.n[b], p,
                                      w.Zgen + P.row_off[b] * p, s));
        Zp = w.Zgen;
    }
    hipLaunchKernelGGL(batch_pack_yz_kernel, dim3(nblocks(rt)), dim3(256), 0, s, y, Zp, P.rows, p, w.Bm);
    B_CHECK(hipGetLastError());

    std::vector<BProb> probs;
    std::vector<BTile> queue;
    int ntiles = 0;
    if (P.tile_j == 0) {
        if (P.tune) {
            int st = tune_tiles(P, w, w.Bm, s);
            if (st != MFGP_OK) return st;
        } else {
            P.tile_j = kDefaultTile;
        }
    }
    {
        int st = upload_tiles(P, w, P.tile_j, ntiles, probs, queue, s);
        if (st != MFGP_OK) return st;
    }

    using clock = std::chrono::steady_clock;
    auto t0 = clock::now();
    // CG state
    CgState st;
    st.x = w.X64;
    st.r = w.R;
    st.p = w.P;
    st.ap = w.AP;
    st.rr = w.scal;
    st.bnorm2 = w.scal + T;
    st.pap = w.scal + 2 * T;
    st.alpha = w.scal + 3 * T;
    st.beta = w.scal + 4 * T;
    st.rrn = w.scal + 7 * T;
    st.active = w.ints;
    st.status = w.ints + T;
    st.iters = w.ints + 2 * T;
    st.lanlen = w.ints + 3 * T;
    st.coeff = w.coeff;
    int* restart = w.ints + 4 * T;

    B_CHECK(bdots_ff(P, w, w.Bm, w.Bm, st.bnorm2, s));
    B_CHECK(fill_f64(st.x, rt, 0.0, s));
    B_CHECK(copy2_f32(w.Bm, st.r, st.p, rt, s));
    B_CHECK(bdots_ff(P, w, st.r, st.r, st.rr, s));
    hipLaunchKernelGGL(bcg_init_kernel, dim3(nblocks(T)), dim3(256), 0, s, st, T, tol * tol);
    const std::vector<int> log_on(T, 1);
    B_CHECK(hipMemcpyAsync(w.logflag, log_on.data(), T * sizeof(int), hipMemcpyHostToDevice, s));

    int check_every = opts->check_every > 0 ? opts->check_every : 8;
    // Residual replacement only with a check at least every other iteration
    // (as in the single-problem solver); the default graph of 8 iterations
    // runs plain cycles with refinement.
    const bool may_replace = !opts->no_replacement && check_every <= kMaxReplaceGap;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    P.graph_launches = 0;
    if (P.use_graph) {
        B_CHECK(hipStreamSynchronize(s));
        if (!P.cap_stream) B_CHECK(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking));
        hipStream_t cs = P.cap_stream;
        B_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        timing_suspend(true);   // no event records inside the graph
        hipError_t ce = hipSuccess;
        for (int k = 0; k < check_every && ce == hipSuccess; ++k) ce = batch_iteration(P, w, st, ntiles, tol, cs);
        timing_suspend(false);
        hipError_t ee = hipStreamEndCapture(cs, &graph);
        if (ce != hipSuccess || ee != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            set_last_hip_error(ce != hipSuccess ? ce : ee);
            return MFGP_ERR_HIP;
        }
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(graph);
            set_last_hip_error(ie);
            return MFGP_ERR_HIP;
        }
    }
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    };
#define B_CHECK2(expr)                         \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) {                \
            cleanup();                         \
            set_last_hip_error(e_);            \
            return MFGP_ERR_HIP;               \
        }                                      \
    } while (0)

    std::vector<int> h_active(T), h_iters(T), h_status(T), h_restart(T), h_refine(T, 0), h_lan(T);
    std::vector<double> h_relt(T), h_rr(T), h_b2(T), h_rep(T), h_cross(T);
    std::vector<int> h_norepl(T, 0), h_nrep(T, 0), h_skips(T, 0);
    // stagnation (stall.hpp): a stagnated cycle ends and is refined (the
    // batched sweep keeps its precision: no fallback to another form)
    std::vector<StallTracker> h_stall(T);
    std::vector<int> h_nstall(T, 0);
    // per problem: finished (every column assessed and stopped); per column:
    // stopped and judged final since its last restart, and its last
    // recomputed true relative residual
    std::vector<char> done(nprob, 0), assessed(T, 0);
    std::vector<double> h_final(T, 0.0);
    B_CHECK2(hipMemcpyAsync(h_rep.data(), st.rr, T * sizeof(double), hipMemcpyDeviceToHost, s));
    B_CHECK2(hipMemcpyAsync(h_b2.data(), st.bnorm2, T * sizeof(double), hipMemcpyDeviceToHost, s));
    B_CHECK2(hipStreamSynchronize(s));
    for (int q = 0; q < T; ++q) h_stall[q].begin(0, h_rep[q]);
    // quadratures of finished problems, overlapped with the rest of the solve
    SlqQueue slq(T);
    std::vector<char> queued(T, 0);
    slq.zn = h_b2;   // ||z_q||^2 (the column norms of B, computed once)
    {
        // at most 16 threads: they run beside the thread that drives the GPU,
        // and a larger host count need not be this process's CPU share
        const unsigned hw = std::thread::hardware_concurrency();
        slq.start(static_cast<int>(std::max(1u, std::min(hw ? hw : 1u, 16u))));
    }
    // copy the Lanczos coefficients of the probe columns of the listed
    // problems (their columns no longer iterate) and queue their quadratures
    auto queue_slq = [&](const std::vector<int>& probs_done) -> hipError_t {
        hipError_t e = hipMemcpyAsync(h_lan.data(), st.lanlen, T * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        std::vector<int> qs_new;
        for (int b : probs_done)
            for (int c = 1; c < t && e == hipSuccess; ++c) {
                const int q = b * t + c;
                if (queued[q]) continue;
                slq.len[q] = h_lan[q];
                if (h_lan[q] >= 1) {
                    slq.cf[q].resize(2 * static_cast<size_t>(h_lan[q]));
                    e = hipMemcpyAsync(slq.cf[q].data(), w.coeff + static_cast<size_t>(q) * max_iter * 2,
                                       2 * h_lan[q] * sizeof(double), hipMemcpyDeviceToHost, s);
                }
                qs_new.push_back(q);
            }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        for (int q : qs_new) {
            queued[q] = 1;
            slq.push(q);
        }
        return hipSuccess;
    };
    const int report_every = opts->progress_every > 0 ? opts->progress_every : 100;
    int next_report = report_every;
    int steps = 0;   // iterations run by the solver (every cycle; all columns advance together)
    for (;;) {
        B_CHECK2(hipMemcpyAsync(h_active.data(), st.active, T * sizeof(int), hipMemcpyDeviceToHost, s));
        B_CHECK2(hipMemcpyAsync(h_iters.data(), st.iters, T * sizeof(int), hipMemcpyDeviceToHost, s));
        B_CHECK2(hipMemcpyAsync(h_rr.data(), st.rr, T * sizeof(double), hipMemcpyDeviceToHost, s));
        B_CHECK2(hipStreamSynchronize(s));
        bool stop = false;
        for (int q = 0; q < T; ++q) {
            if (!h_active[q] || h_iters[q] >= max_iter) continue;
            if (h_stall[q].update(h_iters[q], h_rr[q])) {
                h_active[q] = 0;
                h_nstall[q] += 1;
                stop = true;
            }
        }
        if (stop)
            B_CHECK2(hipMemcpyAsync(st.active, h_active.data(), T * sizeof(int), hipMemcpyHostToDevice, s));

        // A column that has stopped ends its cycle now, not when the slowest
        // problem of the batch (or the slowest column of its own problem)
        // does: its problem's true residual is recomputed (FP64 accumulation)
        // and the column restarts from it if it is above tol, while every
        // other column keeps iterating.
        std::vector<int> ending;
        for (int b = 0; b < nprob; ++b) {
            if (done[b]) continue;
            bool fresh = false;
            for (int c = 0; c < t; ++c) {
                const int q = b * t + c;
                fresh = fresh || (!(h_active[q] && h_iters[q] < max_iter) && !assessed[q]);
            }
            if (fresh) ending.push_back(b);
        }
        if (!ending.empty()) {
            std::vector<int> newly_done;
            for (int b : ending) {
                const int64_t o = P.row_off[b] * t;
                B_CHECK2(residual_f64(ops[b], w.Bm + o, st.x + o, t, w.R64 + o, w.resid, s));
            }
            // columns of every problem are reduced; only those of the ending
            // problems (whose R64 was just written) are read
            B_CHECK2(bdots_dd(P, w, w.R64, w.R64, w.tmp, s));
            B_CHECK2(hipMemcpyAsync(h_relt.data(), w.tmp, T * sizeof(double), hipMemcpyDeviceToHost, s));
            B_CHECK2(hipMemcpyAsync(h_status.data(), st.status, T * sizeof(int), hipMemcpyDeviceToHost, s));
            B_CHECK2(hipStreamSynchronize(s));
            std::fill(h_restart.begin(), h_restart.end(), 0);
            bool again = false;
            for (int b : ending) {
                bool finished = true;
                for (int c = 0; c < t; ++c) {
                    const int q = b * t + c;
                    if (h_active[q] && h_iters[q] < max_iter) {
                        finished = false;   // still iterating: its R64 is not read
                        continue;
                    }
                    if (assessed[q]) continue;
                    h_final[q] = h_b2[q] > 0.0 ? std::sqrt(h_relt[q] / h_b2[q]) : 0.0;
                    const bool need = h_status[q] == MFGP_OK && !(h_final[q] <= tol) && std::isfinite(h_final[q]) &&
                                      h_refine[q] < max_refine && h_iters[q] < max_iter;
                    if (need) {
                        h_restart[q] = 1;
                        h_refine[q] += 1;
                        finished = false;
                        again = true;
                    } else {
                        assessed[q] = 1;
                    }
                }
                if (finished) {
                    done[b] = 1;
                    newly_done.push_back(b);
                }
            }
            if (again) {
                B_CHECK2(hipMemcpyAsync(restart, h_restart.data(), T * sizeof(int), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(bcg_restart_kernel, dim3(static_cast<unsigned>(P.segs.size())), dim3(256), 0, s,
                                   st, w.segs, t, w.R64, restart);
                B_CHECK2(bdots_ff(P, w, st.r, st.r, w.tmp + T, s));
                hipLaunchKernelGGL(bcg_activate_kernel, dim3(nblocks(T)), dim3(256), 0, s, st, T, restart,
                                   w.tmp + T, w.logflag);
                B_CHECK2(hipGetLastError());
                B_CHECK2(hipMemcpyAsync(h_rep.data(), w.tmp + T, T * sizeof(double), hipMemcpyDeviceToHost, s));
                B_CHECK2(hipStreamSynchronize(s));
                for (int q = 0; q < T; ++q) {
                    if (!h_restart[q]) continue;
                    h_norepl[q] = 0;   // a fresh cycle starts without drift
                    h_stall[q].begin(h_iters[q], h_rep[q]);
                    h_active[q] = h_rep[q] > 0.0 ? 1 : 0;
                    h_rr[q] = h_rep[q];
                    if (!h_active[q]) assessed[q] = 1;   // restarted at an exact zero residual
                }
            }
            if (!newly_done.empty()) B_CHECK2(queue_slq(newly_done));
        }

        // Residual replacement (as in the single-problem solver): a tenfold drop
        // since the last true residual triggers it; active columns that fell at
        // least 1.5x join; only problems with a flagged column recompute.
        // Triggers and joiners are per problem, exactly as in the single-problem
        // solver, so a problem's replacements do not depend on the others.
        bool any = false, replace = false;
        std::vector<char> trig(nprob, 0);
        for (int q = 0; q < T; ++q) {
            const bool act = h_active[q] && h_iters[q] < max_iter;
            any = any || act;
            const bool can = act && !h_norepl[q] && may_replace;
            if (can && h_rr[q] <= 0.01 * h_rep[q]) trig[q / t] = 1;
            h_restart[q] = (can && h_rr[q] <= 0.44 * h_rep[q]) ? 1 : 0;
        }
        if (!any) break;   // every problem is done
        for (int q = 0; q < T; ++q) h_restart[q] = trig[q / t] ? h_restart[q] : 0;
        for (int b = 0; b < nprob; ++b) replace = replace || trig[b];
        if (replace) {
            for (int b = 0; b < nprob; ++b) {
                if (!trig[b]) continue;
                const int64_t o = P.row_off[b] * t;
                B_CHECK2(residual_f64(ops[b], w.Bm + o, st.x + o, t, w.R64 + o, w.resid, s));
            }
            // drift of the recomputed problems (others are not read):
            // |r_true - r_rec|^2 = |r_true|^2 + |r_rec|^2 - 2 r_true^T r_rec
            B_CHECK2(bdots_dd(P, w, w.R64, w.R64, w.tmp, s));
            B_CHECK2(bdots_df(P, w, w.R64, st.r, w.tmp + 2 * T, s));
            B_CHECK2(hipMemcpyAsync(h_relt.data(), w.tmp, T * sizeof(double), hipMemcpyDeviceToHost, s));
            B_CHECK2(hipMemcpyAsync(h_cross.data(), w.tmp + 2 * T, T * sizeof(double), hipMemcpyDeviceToHost, s));
            B_CHECK2(hipStreamSynchronize(s));
            for (int q = 0; q < T; ++q) {
                if (!h_restart[q]) continue;
                const double drift2 = h_relt[q] + h_rr[q] - 2.0 * h_cross[q];
                if (!(drift2 <= kMaxDrift2 * h_relt[q])) {
                    h_restart[q] = 0;     // run this cycle out and refine instead
                    h_norepl[q] = 1;
                    h_skips[q] += 1;
                } else {
                    h_nrep[q] += 1;
                }
            }
            B_CHECK2(hipMemcpyAsync(restart, h_restart.data(), T * sizeof(int), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(bcg_replace_kernel, dim3(static_cast<unsigned>(P.segs.size())), dim3(256), 0, s, st,
                               w.segs, t, w.R64, restart);
            B_CHECK2(bdots_ff(P, w, st.r, st.r, w.tmp + T, s));
            hipLaunchKernelGGL(bcg_set_rr_kernel, dim3(nblocks(T)), dim3(256), 0, s, st, T, restart, w.tmp + T);
            B_CHECK2(hipMemcpyAsync(h_rr.data(), st.rr, T * sizeof(double), hipMemcpyDeviceToHost, s));
            B_CHECK2(hipStreamSynchronize(s));
            for (int q = 0; q < T; ++q)
                if (h_restart[q]) h_rep[q] = h_rr[q];
        }
        if (opts->progress && steps >= next_report) {
            opts->progress(opts->progress_user, steps, worst_recurrence(h_active, h_rr, h_b2));
            while (next_report <= steps) next_report += report_every;
        }
        steps += check_every;
        if (exec) {
            B_CHECK2(hipGraphLaunch(exec, s));
            P.graph_launches += 1;
        } else {
            for (int k = 0; k < check_every; ++k) B_CHECK2(batch_iteration(P, w, st, ntiles, tol, s));
        }
    }
    B_CHECK2(hipMemcpyAsync(h_status.data(), st.status, T * sizeof(int), hipMemcpyDeviceToHost, s));
    for (int q = 0; q < T; ++q) h_relt[q] = h_final[q];
    cleanup();
    B_CHECK(hipMemcpyAsync(h_rr.data(), st.rr, T * sizeof(double), hipMemcpyDeviceToHost, s));
    B_CHECK(hipMemcpyAsync(h_lan.data(), st.lanlen, T * sizeof(int), hipMemcpyDeviceToHost, s));
    B_CHECK(hipMemcpyAsync(h_iters.data(), st.iters, T * sizeof(int), hipMemcpyDeviceToHost, s));
    B_CHECK(hipStreamSynchronize(s));
    int worst = MFGP_OK;
    std::vector<mfgp_cg_info> inf(T);
    for (int q = 0; q < T; ++q) {
        int sq = h_status[q];
        if (sq == MFGP_OK && !(h_relt[q] <= tol)) sq = MFGP_NOT_CONVERGED;
        if (sq == MFGP_BREAKDOWN) worst = MFGP_BREAKDOWN;
        else if (sq == MFGP_NOT_CONVERGED && worst == MFGP_OK) worst = MFGP_NOT_CONVERGED;
        inf[q].iters = h_iters[q];
        inf[q].lanczos_len = h_lan[q];
        inf[q].refinements = h_refine[q];
        inf[q].status = sq;
        inf[q].rel_resid_recurrence = h_b2[q] > 0.0 ? std::sqrt(h_rr[q] / h_b2[q]) : 0.0;
        inf[q].rel_resid_true = h_relt[q];
        inf[q].replacements = h_nrep[q];
        inf[q].drift_skips = h_skips[q];
        inf[q].stalls = h_nstall[q];
        inf[q].precision = opts->precision;
    }
    if (info) std::memcpy(info, inf.data(), T * sizeof(mfgp_cg_info));
    timing_phase(0, std::chrono::duration<double, std::milli>(clock::now() - t0).count());
    t0 = clock::now();

    // Column dot products (x^T b for the data fit) and the quadratures.
    double* xb = w.tmp + T;
    double* xx = w.tmp + 2 * T;
    B_CHECK(bdots_df(P, w, w.X64, w.Bm, xb, s));
    B_CHECK(bdots_dd(P, w, w.X64, w.X64, xx, s));
    std::vector<double> h(3 * T);
    B_CHECK(hipMemcpyAsync(h.data() + T, xb, 2 * T * sizeof(double), hipMemcpyDeviceToHost, s));
    // the problems whose quadratures are not queued yet (those that ended
    // with the solve; queue_slq synchronises the stream, also for h), then
    // every quadrature
    {
        std::vector<int> rest;
        for (int b = 0; b < nprob; ++b)
            for (int c = 1; c < t; ++c)
                if (!queued[b * t + c]) {
                    rest.push_back(b);
                    break;
                }
        B_CHECK(queue_slq(rest));
    }
    slq.finish(false);
    const std::vector<double>& qv = slq.qv;
    const std::vector<int>& qs = slq.qs;
    int slq_status = MFGP_OK;
    const double two_pi = 6.283185307179586477;
    for (int b = 0; b < nprob; ++b) {
        double ld = 0.0;
        for (int c = 1; c < t; ++c) {
            ld += qv[b * t + c];
            if (qs[b * t + c] != MFGP_OK) slq_status = MFGP_BREAKDOWN;
        }
        ld /= p;
        mll[b] = -0.5 * (h[T + b * t] + ld + static_cast<double>(P.n[b]) * std::log(two_pi));
        if (logdet) logdet[b] = ld;
    }
    timing_phase(1, std::chrono::duration<double, std::milli>(clock::now() - t0).count());
    t0 = clock::now();

    if (grad) {
        float* Ag = w.R;
        float* Bg = w.P;
        B_CHECK(f64_to_f32(w.X64, Ag, rt, s));
        B_CHECK(copy2_f32(w.Bm, Bg, Bg, rt, s));
        hipLaunchKernelGGL(batch_set_col0_kernel, dim3(nblocks(P.rows)), dim3(256), 0, s, w.X64, Bg, P.rows, t);
        B_CHECK(hipGetLastError());
        ColW cw{};
        cw.w[0] = 0.5f;
        for (int c = 1; c < t; ++c) cw.w[c] = static_cast<float>(-0.5 / p);
        double* part = reinterpret_cast<double*>(w.part);
        double* sums = part + static_cast<size_t>(ntiles) * kWidth;
        void* tok = timing_begin(s);
        B_CHECK(launch_badj(P.family, t, w, ntiles, Ag, Bg, cw, part, s));
        {
            double ent = 0.0, fl = 0.0;
            for (int b = 0; b < nprob; ++b) {
                const double e2 = static_cast<double>(P.n[b]) * static_cast<double>(P.n[b]);
                ent += e2;
                fl += e2 * sweep_flops_per_entry(P.family, P.kern[b].d, t, true);
            }
            timing_end(tok, s, kSweepAdjoint, ent, fl);
        }
        hipLaunchKernelGGL(adjoint_stage2_kernel, dim3(nblocks(static_cast<int64_t>(nprob) * kWidth)), dim3(256),
                           0, s, part, w.probs, nprob, sums);
        B_CHECK(hipGetLastError());
        std::vector<double> hs(static_cast<size_t>(nprob) * kWidth);
        B_CHECK(hipMemcpyAsync(hs.data(), sums, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        B_CHECK(hipStreamSynchronize(s));
        double* g = grad;
        for (int b = 0; b < nprob; ++b) {
            const Operator& op = ops[b];
            const mfgp_kernel& k = P.kern[b];
            const double* G = hs.data() + static_cast<size_t>(b) * kWidth;
            double shared = 0.0;
            for (int q = 0; q < op.d; ++q) {
                const double gq = static_cast<double>(op.s2) * lengthscale_factor_b(op.family, op.ls[q]) * G[q];
                if (k.ard) g[q] = gq;
                else shared += gq;
            }
            const int nl = k.ard ? op.d : 1;
            if (!k.ard) g[0] = shared;
            g[nl] = G[op.d];
            double tr = 0.0;
            for (int c = 1; c < t; ++c) tr += h[T + b * t + c];
            g[nl + 1] = 0.5 * h[2 * T + b * t] - 0.5 * tr / p;
            g += nl + 2;
        }
        timing_phase(2, std::chrono::duration<double, std::milli>(clock::now() - t0).count());
    }
    if (worst != MFGP_OK) return worst;
    return slq_status;
}

}  // extern "C"
