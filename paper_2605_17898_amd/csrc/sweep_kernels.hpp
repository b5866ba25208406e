// Entry-sweep kernels: out_i = sum_j k(u_i, u_j) V_j over a j-range, entries
// generated on the fly and never stored (the fused matrix-free product of
// LightGP Sec. 4.1, Table 3; O(N) memory as in Sec. 2).
//
// Mapping on gfx950.  One lane owns one output row i and keeps u_i and the TB
// accumulators in VGPRs.  The j loop is wave-uniform, so u_j and V_j are read
// with scalar loads into SGPRs and feed the VALU as its scalar operand: no LDS
// staging, no barriers, and every VALU slot goes to entry arithmetic.  The
// j-range of a launch is split into `chunks` ranges (split-j) to fill the 256
// CUs; partial sums are reduced afterwards in a fixed order, so results are
// deterministic.  Block -> (row block, chunk) is XCD-aware: with chunks a
// multiple of 8, all row blocks of one chunk land on the same XCD
// (round-robin dispatch), so that chunk's u_j / V_j stay in that XCD's L2.
#pragma once

#include "common.hpp"

namespace mfgp {

__device__ __forceinline__ void map_block(int b, int chunks, int& rb, int& ch) {
    if ((chunks & 7) == 0) {
        const int xcd = b & 7;
        const int k = b >> 3;
        const int cpx = chunks >> 3;
        ch = xcd + 8 * (k % cpx);
        rb = k / cpx;
    } else {
        ch = b % chunks;
        rb = b / chunks;
    }
}

// j-values per inner accumulation segment (a multiple of every 2 * unroll)
constexpr int kSeg = 256;

// j-values processed per unrolled step: keeps (D + TB) * JU scalar words <= 32.
template <int D, int TB>
constexpr int sweep_unroll() {
    constexpr int w = D + TB;
    return w <= 4 ? 8 : (w <= 8 ? 4 : (w <= 16 ? 2 : 1));
}

// Sums acc[c] = sum_{q < cnt} k(u_i, uc_q) vc[q][c] for one lane's row (u_i in
// VGPRs); uc / vc are wave-uniform, so their elements arrive through scalar
// loads.  Shared by the single-problem and the batched (persistent) sweeps.
template <int FAM, int D, int TB>
__device__ __forceinline__ void sweep_rows(const float (&ui)[D], const float* __restrict__ uc,
                                           const float* __restrict__ vc, int cnt, float (&acc)[TB]) {
#pragma unroll
    for (int c = 0; c < TB; ++c) acc[c] = 0.0f;
    constexpr int JU = sweep_unroll<D, TB>();
    const int cmain = cnt - cnt % (2 * JU);   // main loop: whole A/B step pairs

    // Two-level accumulation: acc sums one segment of kSeg j's, tot sums the
    // segments, so no FP32 running sum is longer than max(kSeg, cnt / kSeg).
    float tot[TB];
#pragma unroll
    for (int c = 0; c < TB; ++c) tot[c] = 0.0f;

    // Ping-pong software pipeline over two SGPR sets A and B: the scalar loads
    // of one set are in flight while the other set's entries are computed, and
    // no register copies are needed between steps.
    float au[JU * D], av[JU * TB], bu[JU * D], bv[JU * TB];
    if (cmain > 0) {
#pragma unroll
        for (int k = 0; k < JU * D; ++k) au[k] = uc[k];
#pragma unroll
        for (int k = 0; k < JU * TB; ++k) av[k] = vc[k];
    }
    for (int seg = 0; seg < cmain; seg += kSeg) {
        const int send = seg + kSeg < cmain ? seg + kSeg : cmain;
        for (int q = seg; q < send; q += 2 * JU) {
            const int qb = q + JU;
#pragma unroll
            for (int k = 0; k < JU * D; ++k) bu[k] = uc[qb * D + k];
#pragma unroll
            for (int k = 0; k < JU * TB; ++k) bv[k] = vc[qb * TB + k];
#pragma unroll
            for (int r = 0; r < JU; ++r) {
                const float e = kentry<FAM>(sqdist<D>(ui, au + r * D));
#pragma unroll
                for (int c = 0; c < TB; ++c) acc[c] = fmaf(e, av[r * TB + c], acc[c]);
            }
            const int qa = q + 2 * JU < cmain ? q + 2 * JU : q;
#pragma unroll
            for (int k = 0; k < JU * D; ++k) au[k] = uc[qa * D + k];
#pragma unroll
            for (int k = 0; k < JU * TB; ++k) av[k] = vc[qa * TB + k];
#pragma unroll
            for (int r = 0; r < JU; ++r) {
                const float e = kentry<FAM>(sqdist<D>(ui, bu + r * D));
#pragma unroll
                for (int c = 0; c < TB; ++c) acc[c] = fmaf(e, bv[r * TB + c], acc[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < TB; ++c) {
            tot[c] += acc[c];
            acc[c] = 0.0f;
        }
    }
    for (int q = cmain; q < cnt; ++q) {
        const float e = kentry<FAM>(sqdist<D>(ui, uc + q * D));
#pragma unroll
        for (int c = 0; c < TB; ++c) acc[c] = fmaf(e, vc[q * TB + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < TB; ++c) acc[c] += tot[c];
}

template <int FAM, int D, int TB>
__global__ __launch_bounds__(kBlock) void sweep_f32_kernel(
    const float* __restrict__ Ur, const float* __restrict__ Uc, const float* __restrict__ V,
    int64_t m, int64_t n, int chunks, int64_t jchunk, float* __restrict__ partial) {
    // V is a packed [n, TB] block (row stride TB), so one scalar load fetches
    // the right-hand sides of several consecutive j.
    int rb, ch;
    map_block(blockIdx.x, chunks, rb, ch);
    const int64_t i = static_cast<int64_t>(rb) * kBlock + threadIdx.x;
    const int64_t ii = i < m ? i : m - 1;
    float ui[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ui[k] = Ur[ii * D + k];
    const int64_t j0 = static_cast<int64_t>(ch) * jchunk;
    const int64_t jend = j0 + jchunk < n ? j0 + jchunk : n;
    const int cnt = j0 < jend ? static_cast<int>(jend - j0) : 0;   // wave-uniform, < 2^31
    float acc[TB];
    sweep_rows<FAM, D, TB>(ui, Uc + j0 * D, V + j0 * TB, cnt, acc);
    if (i < m) {
        float* p = partial + (static_cast<int64_t>(ch) * m + i) * TB;
#pragma unroll
        for (int c = 0; c < TB; ++c) p[c] = acc[c];
    }
}

// Same sweep with the products of the FP32 entries and FP64 right-hand sides
// accumulated in FP64 (an FP32 x FP32 product is exact in FP64; here V is
// FP64 and the entry is widened).  Used for the recomputed CG residual.
template <int FAM, int D, int TB>
__global__ __launch_bounds__(kBlock) void sweep_f64acc_kernel(
    const float* __restrict__ Ur, const float* __restrict__ Uc, const double* __restrict__ V,
    int ldv, int64_t m, int64_t n, int chunks, int64_t jchunk, double* __restrict__ partial) {
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
        const double e = static_cast<double>(kentry<FAM>(sqdist<D>(ui, Uc + j * D)));
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

#define MFGP_TB_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(16) X(17) X(32) X(33)
#define MFGP_TB64_LIST(X) X(1) X(2) X(4) X(8) X(16) X(17) X(32) X(33)

template <int FAM, int D>
hipError_t sweep_f32_fd(int tb, const SweepArgs& a, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.plan.rowblocks) * a.plan.chunks);
    switch (tb) {
#define MFGP_CASE(TBV)                                                                       \
    case TBV:                                                                                \
        hipLaunchKernelGGL((sweep_f32_kernel<FAM, D, TBV>), grid, dim3(kBlock), 0, s, a.Ur, \
                           a.Uc, a.V, a.m, a.n, a.plan.chunks, a.plan.jchunk, a.partial);    \
        return hipGetLastError();
        MFGP_TB_LIST(MFGP_CASE)
#undef MFGP_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <int FAM, int D>
hipError_t sweep_f64_fd(int tb, const SweepArgs64& a, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.plan.rowblocks) * a.plan.chunks);
    switch (tb) {
#define MFGP_CASE(TBV)                                                                          \
    case TBV:                                                                                   \
        hipLaunchKernelGGL((sweep_f64acc_kernel<FAM, D, TBV>), grid, dim3(kBlock), 0, s, a.Ur, \
                           a.Uc, a.V, a.ldv, a.m, a.n, a.plan.chunks, a.plan.jchunk,            \
                           a.partial);                                                          \
        return hipGetLastError();
        MFGP_TB64_LIST(MFGP_CASE)
#undef MFGP_CASE
        default:
            return hipErrorInvalidValue;
    }
}

template <int FAM>
hipError_t sweep_f32_family(int D, int tb, const SweepArgs& a, hipStream_t s) {
    switch (D) {
        case 1: return sweep_f32_fd<FAM, 1>(tb, a, s);
        case 2: return sweep_f32_fd<FAM, 2>(tb, a, s);
        case 3: return sweep_f32_fd<FAM, 3>(tb, a, s);
        case 4: return sweep_f32_fd<FAM, 4>(tb, a, s);
        case 5: return sweep_f32_fd<FAM, 5>(tb, a, s);
        case 6: return sweep_f32_fd<FAM, 6>(tb, a, s);
        case 7: return sweep_f32_fd<FAM, 7>(tb, a, s);
        case 8: return sweep_f32_fd<FAM, 8>(tb, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int FAM>
hipError_t sweep_f64_family(int D, int tb, const SweepArgs64& a, hipStream_t s) {
    switch (D) {
        case 1: return sweep_f64_fd<FAM, 1>(tb, a, s);
        case 2: return sweep_f64_fd<FAM, 2>(tb, a, s);
        case 3: return sweep_f64_fd<FAM, 3>(tb, a, s);
        case 4: return sweep_f64_fd<FAM, 4>(tb, a, s);
        case 5: return sweep_f64_fd<FAM, 5>(tb, a, s);
        case 6: return sweep_f64_fd<FAM, 6>(tb, a, s);
        case 7: return sweep_f64_fd<FAM, 7>(tb, a, s);
        case 8: return sweep_f64_fd<FAM, 8>(tb, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mfgp
