// Column-wise vector kernels for CG on [n, t] row-major blocks: FP64 dot
// products, the fused CG updates and the FP64 scalar steps.
//
// Reductions are "striped": with S = floor(G * 256 / t) * t threads, thread k
// walks elements k, k + S, k + 2S, ... which all belong to column k mod t, so
// every load is coalesced and each thread accumulates one column in FP64.
// Block and grid sums then run in a fixed order, so results are bitwise
// reproducible.
#include "common.hpp"
#include "internal.hpp"
#include "vec.hpp"

namespace mfgp {

int stripe_blocks(int64_t n, int t) {
    const int64_t total = n * t;
    int64_t g = (total + 255) / 256;
    if (g > 512) g = 512;
    const int64_t need = (t + 255) / 256;  // at least t threads
    if (g < need) g = need;
    return static_cast<int>(g);
}

__device__ __forceinline__ double block_column_sum(const double* lds, int t, int c,
                                                   int64_t block_first) {
    // Sum over this block's threads whose column equals c; thread tid has
    // column (block_first + tid) mod t.
    const int off = static_cast<int>(block_first % t);
    int tid0 = c - off;
    if (tid0 < 0) tid0 += t;
    double s = 0.0;
    for (int q = tid0; q < 256; q += t) s += lds[q];
    return s;
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void dot_stage1(const TA* __restrict__ a, const TB* __restrict__ b,
                                                  int64_t total, int t, int64_t S,
                                                  double* __restrict__ part) {
    __shared__ double lds[256];
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    double acc = 0.0;
    if (k < S)
        for (int64_t idx = k; idx < total; idx += S)
            acc = fma(static_cast<double>(a[idx]), static_cast<double>(b[idx]), acc);
    lds[threadIdx.x] = (k < S) ? acc : 0.0;
    __syncthreads();
    const int64_t first = static_cast<int64_t>(blockIdx.x) * 256;
    for (int c = threadIdx.x; c < t; c += 256)
        part[static_cast<int64_t>(blockIdx.x) * t + c] = block_column_sum(lds, t, c, first);
}

// One block per column: thread k sums partials k, k + 256, ... in order, then a
// fixed LDS tree combines the 256 thread sums (deterministic).
__global__ __launch_bounds__(256) void dot_stage2(const double* __restrict__ part, int G, int t,
                                                  double* __restrict__ out) {
    __shared__ double lds[256];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) s += part[static_cast<int64_t>(g) * t + c];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = lds[0];
}

// The column sum of dot_stage2 (same order), left in lds[0] of block c.
__device__ __forceinline__ double stage2_sum(const double* __restrict__ part, int G, int t, int c,
                                             double* lds) {
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) s += part[static_cast<int64_t>(g) * t + c];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    return lds[0];
}

// p^T A p of column c (block c) and then its step length alpha = r^T r / p^T A p
// (breakdown when p^T A p is not positive and finite), in one launch: the
// iteration's chain of dependent small kernels is what bounds small solves.
__global__ __launch_bounds__(256) void pap_alpha_kernel(const double* __restrict__ part, int G, CgState st,
                                                        int t) {
    __shared__ double lds[256];
    const int c = blockIdx.x;
    const double pap = stage2_sum(part, G, t, c, lds);
    if (threadIdx.x != 0) return;
    st.pap[c] = pap;
    double a = 0.0;
    if (st.active[c]) {
        if (!(pap > 0.0) || !isfinite(pap) || !isfinite(st.rr[c])) {
            st.status[c] = MFGP_BREAKDOWN;
            st.active[c] = 0;
        } else {
            a = st.rr[c] / pap;
        }
    }
    st.alpha[c] = a;
}

size_t dots_scratch_doubles(int64_t n, int t) {
    return static_cast<size_t>(stripe_blocks(n, t)) * t + 64;
}

template <typename TA, typename TB>
static hipError_t col_dots(const TA* a, const TB* b, int64_t n, int t, double* out,
                           double* scratch, hipStream_t s) {
    const int G = stripe_blocks(n, t);
    const int64_t S = (static_cast<int64_t>(G) * 256 / t) * t;
    hipLaunchKernelGGL((dot_stage1<TA, TB>), dim3(G), dim3(256), 0, s, a, b, n * t, t, S, scratch);
    hipLaunchKernelGGL(dot_stage2, dim3(t), dim3(256), 0, s, scratch, G, t, out);
    return hipGetLastError();
}

hipError_t col_dots_ff(const float* a, const float* b, int64_t n, int t, double* out,
                       double* scratch, hipStream_t s) {
    return col_dots(a, b, n, t, out, scratch, s);
}
hipError_t col_dots_dd(const double* a, const double* b, int64_t n, int t, double* out,
                       double* scratch, hipStream_t s) {
    return col_dots(a, b, n, t, out, scratch, s);
}
hipError_t col_dots_df(const double* a, const float* b, int64_t n, int t, double* out,
                       double* scratch, hipStream_t s) {
    return col_dots(a, b, n, t, out, scratch, s);
}

// ---------------------------------------------------------------- CG steps

// x += alpha p (FP64), r -= alpha Ap (FP32), and striped partial sums of r^2.
__global__ __launch_bounds__(256) void cg_update_kernel(CgState st, int64_t total, int t,
                                                        int64_t S, double* __restrict__ part) {
    __shared__ double lds[256];
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    double acc = 0.0;
    if (k < S) {
        const int c = static_cast<int>(k % t);
        const double a = st.alpha[c];
        const float af = static_cast<float>(a);
        if (a != 0.0) {
            for (int64_t idx = k; idx < total; idx += S) {
                st.x[idx] = fma(a, static_cast<double>(st.p[idx]), st.x[idx]);
                const float r = fmaf(-af, st.ap[idx], st.r[idx]);
                st.r[idx] = r;
                acc = fma(static_cast<double>(r), static_cast<double>(r), acc);
            }
        } else {
            // frozen column: leave x and r untouched (no 0 * inf / NaN)
            for (int64_t idx = k; idx < total; idx += S) {
                const float r = st.r[idx];
                acc = fma(static_cast<double>(r), static_cast<double>(r), acc);
            }
        }
    }
    lds[threadIdx.x] = (k < S) ? acc : 0.0;
    __syncthreads();
    const int64_t first = static_cast<int64_t>(blockIdx.x) * 256;
    for (int c = threadIdx.x; c < t; c += 256)
        part[static_cast<int64_t>(blockIdx.x) * t + c] = block_column_sum(lds, t, c, first);
}

// r^T r of column c (block c), then beta = r'^T r' / r^T r, the logged
// (alpha, beta) while the tridiagonal is recorded, the iteration count and
// the stopping rule for that column, in one launch.
__global__ __launch_bounds__(256) void rr_beta_kernel(const double* __restrict__ part, int G, CgState st, int t,
                                                      double tol2, int log_coeffs, int max_iter) {
    __shared__ double lds[256];
    const int c = blockIdx.x;
    const double rrn = stage2_sum(part, G, t, c, lds);
    if (threadIdx.x != 0) return;
    st.rrn[c] = rrn;
    double b = 0.0;
    if (st.active[c]) {
        b = rrn / st.rr[c];
        if (log_coeffs && st.coeff && st.lanlen[c] < max_iter) {
            double* cf = st.coeff + (static_cast<int64_t>(c) * max_iter + st.lanlen[c]) * 2;
            cf[0] = st.alpha[c];
            cf[1] = b;
            st.lanlen[c] += 1;
        }
        st.iters[c] += 1;
        st.rr[c] = rrn;
        if (!isfinite(rrn)) {
            st.status[c] = MFGP_BREAKDOWN;
            st.active[c] = 0;
        } else if (rrn <= tol2 * st.bnorm2[c] || st.iters[c] >= max_iter) {
            st.active[c] = 0;
        }
    }
    st.beta[c] = b;
}

// p = r + beta p
__global__ void cg_p_kernel(CgState st, int64_t total, int t) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = static_cast<int>(idx % t);
    if (!st.active[c]) return;
    st.p[idx] = fmaf(static_cast<float>(st.beta[c]), st.p[idx], st.r[idx]);
}

// Restart of selected columns from a recomputed FP64 residual:
// r = fl32(R64), p = r for columns with restart[c] set.
__global__ void cg_restart_kernel(CgState st, const double* __restrict__ R64, int64_t total, int t,
                                  const int* __restrict__ restart) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = static_cast<int>(idx % t);
    if (!restart[c]) return;
    const float r = static_cast<float>(R64[idx]);
    st.r[idx] = r;
    st.p[idx] = r;
}

// Residual replacement for flagged columns: r_new = fl32(R64).  The direction
// was already formed from the old residual (p = r_old + beta p_prev); it is
// re-formed as p = r_new + beta p_prev (p += r_new - r_old), so that the next
// step length rr / p^T A p matches r_new.  The host flags only columns whose
// recurrence still agrees with the true residual (small drift).
__global__ void cg_replace_kernel(CgState st, const double* __restrict__ R64, int64_t total, int t,
                                  const int* __restrict__ flag) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    if (flag[idx % t]) {
        const float rn = static_cast<float>(R64[idx]);
        st.p[idx] += rn - st.r[idx];
        st.r[idx] = rn;
    }
}

__global__ void cg_set_rr_kernel(CgState st, int t, const int* __restrict__ flag,
                                 const double* __restrict__ rr_new) {
    for (int c = threadIdx.x; c < t; c += blockDim.x)
        if (flag[c]) st.rr[c] = rr_new[c];
}

// Re-activate restarted columns with their new residual norm.
__global__ void cg_activate_kernel(CgState st, int t, const int* __restrict__ restart,
                                   const double* __restrict__ rr_new) {
    for (int c = threadIdx.x; c < t; c += blockDim.x) {
        if (restart[c]) {
            st.active[c] = rr_new[c] > 0.0 ? 1 : 0;
            st.rr[c] = rr_new[c];
        }
    }
}

__global__ void fill_f64_kernel(double* __restrict__ x, int64_t total, double v) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < total) x[idx] = v;
}

__global__ void copy_f32_kernel(const float* __restrict__ src, float* __restrict__ a,
                                float* __restrict__ b, int64_t total) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < total) {
        a[idx] = src[idx];
        b[idx] = src[idx];
    }
}

__global__ void f64_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                  int64_t total) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < total) dst[idx] = static_cast<float>(src[idx]);
}

static inline unsigned nblk(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

// var[q] = s2 - sum_c Z[q][c] Q[q][c] / sum_c Z[q][c]^2 (FP64 sums; 0 probe
// weight gives the prior s2).
__global__ void diag_variance_kernel(const float* __restrict__ Z, const float* __restrict__ Q, int64_t m, int p,
                                     double s2, float* __restrict__ var) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= m) return;
    double num = 0.0, den = 0.0;
    for (int c = 0; c < p; ++c) {
        const double z = static_cast<double>(Z[q * p + c]);
        num = fma(z, static_cast<double>(Q[q * p + c]), num);
        den = fma(z, z, den);
    }
    var[q] = static_cast<float>(den > 0.0 ? s2 - num / den : s2);
}

hipError_t cg_update_and_beta(const CgState& st, int64_t n, int t, double* scratch, double tol,
                              int log_coeffs, int max_iter, hipStream_t s) {
    const int G = stripe_blocks(n, t);
    const int64_t S = (static_cast<int64_t>(G) * 256 / t) * t;
    hipLaunchKernelGGL(cg_update_kernel, dim3(G), dim3(256), 0, s, st, n * t, t, S, scratch);
    hipLaunchKernelGGL(rr_beta_kernel, dim3(t), dim3(256), 0, s, scratch, G, st, t, tol * tol, log_coeffs,
                       max_iter);
    hipLaunchKernelGGL(cg_p_kernel, dim3(nblk(n * t)), dim3(256), 0, s, st, n * t, t);
    return hipGetLastError();
}

hipError_t cg_pap_alpha(const CgState& st, int64_t n, int t, double* scratch, hipStream_t s) {
    const int G = stripe_blocks(n, t);
    const int64_t S = (static_cast<int64_t>(G) * 256 / t) * t;
    hipLaunchKernelGGL((dot_stage1<float, float>), dim3(G), dim3(256), 0, s, st.p, st.ap, n * t, t, S, scratch);
    hipLaunchKernelGGL(pap_alpha_kernel, dim3(t), dim3(256), 0, s, scratch, G, st, t);
    return hipGetLastError();
}

hipError_t cg_update_rr(const CgState& st, int64_t n, int t, double* scratch, double* rr_out, hipStream_t s) {
    const int G = stripe_blocks(n, t);
    const int64_t S = (static_cast<int64_t>(G) * 256 / t) * t;
    hipLaunchKernelGGL(cg_update_kernel, dim3(G), dim3(256), 0, s, st, n * t, t, S, scratch);
    hipLaunchKernelGGL(dot_stage2, dim3(t), dim3(256), 0, s, scratch, G, t, rr_out);
    return hipGetLastError();
}

hipError_t cg_restart(const CgState& st, const double* R64, int64_t n, int t, const int* restart,
                      hipStream_t s) {
    hipLaunchKernelGGL(cg_restart_kernel, dim3(nblk(n * t)), dim3(256), 0, s, st, R64, n * t, t,
                       restart);
    return hipGetLastError();
}

hipError_t cg_activate(const CgState& st, int t, const int* restart, const double* rr_new,
                       hipStream_t s) {
    hipLaunchKernelGGL(cg_activate_kernel, dim3(1), dim3(256), 0, s, st, t, restart, rr_new);
    return hipGetLastError();
}

hipError_t cg_replace(const CgState& st, const double* R64, int64_t n, int t, const int* flag,
                      double* scratch, double* rr_tmp, hipStream_t s) {
    hipLaunchKernelGGL(cg_replace_kernel, dim3(nblk(n * t)), dim3(256), 0, s, st, R64, n * t, t, flag);
    hipError_t e = col_dots_ff(st.r, st.r, n, t, rr_tmp, scratch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cg_set_rr_kernel, dim3(1), dim3(256), 0, s, st, t, flag, rr_tmp);
    return hipGetLastError();
}

hipError_t fill_f64(double* x, int64_t total, double v, hipStream_t s) {
    hipLaunchKernelGGL(fill_f64_kernel, dim3(nblk(total)), dim3(256), 0, s, x, total, v);
    return hipGetLastError();
}

hipError_t copy2_f32(const float* src, float* a, float* b, int64_t total, hipStream_t s) {
    hipLaunchKernelGGL(copy_f32_kernel, dim3(nblk(total)), dim3(256), 0, s, src, a, b, total);
    return hipGetLastError();
}

hipError_t diag_variance(const float* Z, const float* Q, int64_t m, int p, double s2, float* var, hipStream_t s) {
    hipLaunchKernelGGL(diag_variance_kernel, dim3(nblk(m)), dim3(256), 0, s, Z, Q, m, p, s2, var);
    return hipGetLastError();
}

hipError_t f64_to_f32(const double* src, float* dst, int64_t total, hipStream_t s) {
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nblk(total)), dim3(256), 0, s, src, dst, total);
    return hipGetLastError();
}

}  // namespace mfgp
