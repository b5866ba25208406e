// C-ABI entry points (declared in include/mfgp.h): argument validation on the
// host, workspace carving, and orchestration of the kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "cg.hpp"
#include "vec.hpp"
#include "precond.hpp"
#include "internal.hpp"

namespace mfgp {

static thread_local int g_last_hip = 0;
void set_last_hip_error(hipError_t e) { g_last_hip = static_cast<int>(e); }

int slq_quadrature(const double* coeffs, int m, double znorm2, double* q);

// ---------------------------------------------------------------- small kernels

__global__ void pack_yz_kernel(const float* __restrict__ y, const float* __restrict__ Z, int64_t n,
                               int p, float* __restrict__ out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int t = p + 1;
    if (idx >= n * t) return;
    const int64_t i = idx / t;
    const int c = static_cast<int>(idx % t);
    out[idx] = c == 0 ? y[i] : Z[i * p + (c - 1)];
}

// dst[i * t] = fl32(src[i * t])  (column 0 of an [n, t] block)
__global__ void set_col0_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n,
                                int t) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i * t] = static_cast<float>(src[i * t]);
}

__global__ void copy_col0_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                                 int t) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i * t];
}

// SplitMix64 (Steele, Lea & Flood 2014): output k of the stream seeded with s
// is mix(s + k * 0x9E3779B97F4A7C15); entry (j, c) uses k = c n + j + 1.
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void rademacher_kernel(uint64_t seed, int64_t n, int p, float* __restrict__ Z) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * p) return;
    const int64_t j = idx / p;
    const int64_t c = idx % p;
    const uint64_t k = static_cast<uint64_t>(c) * static_cast<uint64_t>(n) + static_cast<uint64_t>(j) + 1ull;
    const uint64_t z = splitmix_mix(seed + k * 0x9E3779B97F4A7C15ull);
    Z[idx] = (z >> 63) ? -1.0f : 1.0f;
}

hipError_t launch_rademacher(uint64_t seed, int64_t n, int p, float* Z, hipStream_t s) {
    const int64_t total = n * p;
    hipLaunchKernelGGL(rademacher_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                       0, s, seed, n, p, Z);
    return hipGetLastError();
}

static inline unsigned nb(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

// ---------------------------------------------------------------- validation

static bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

// A product term: factors of any family, at most one periodic, within
// MFGP_MAX_D features in all (d per RBF, Matern or Linear factor, 2d for the
// periodic one).
static int check_product(const mfgp_kernel* k, int d) {
    int nf = 0, nper = 0, feats = 0;
    for (const mfgp_kernel* q = k; q; q = q->times) {
        if (++nf > MFGP_MAX_TERMS) return MFGP_UNSUPPORTED;
        if (q->family < MFGP_RBF || q->family > MFGP_LINEAR) return MFGP_ERR_ARG;
        if (q->d != d) return MFGP_ERR_ARG;
        if (q->family == MFGP_PERIODIC) {
            if (!finite_pos(q->period)) return MFGP_ERR_ARG;
            ++nper;
            feats += 2 * d;
        } else {
            feats += d;
        }
        if (q->family == MFGP_LINEAR) continue;
        const int nl = q->ard ? d : 1;
        for (int j = 0; j < nl; ++j)
            if (!finite_pos(q->lengthscale[j])) return MFGP_ERR_ARG;
    }
    if (nper > 1 || feats > MFGP_MAX_D) return MFGP_UNSUPPORTED;
    if (!finite_pos(k->outputscale)) return MFGP_ERR_ARG;
    return MFGP_OK;
}

// One term of a kernel (the head's d is every term's d).
static int check_term(const mfgp_kernel* k, int d) {
    if (k->times) return check_product(k, d);
    if (k->family < MFGP_RBF || k->family > MFGP_LINEAR) return MFGP_ERR_ARG;
    if (k->d != d) return MFGP_ERR_ARG;
    if (k->family == MFGP_PERIODIC) {
        if (!finite_pos(k->period)) return MFGP_ERR_ARG;
        if (2 * k->d > MFGP_MAX_D) return MFGP_UNSUPPORTED;   // 2 d circle features
    }
    if (k->family != MFGP_LINEAR) {
        const int nl = k->ard ? k->d : 1;
        for (int q = 0; q < nl; ++q)
            if (!finite_pos(k->lengthscale[q])) return MFGP_ERR_ARG;
    }
    if (!finite_pos(k->outputscale)) return MFGP_ERR_ARG;
    return MFGP_OK;
}

static int check_kernel(const mfgp_kernel* k, bool need_noise) {
    if (!k) return MFGP_ERR_ARG;
    if (k->d < 1) return MFGP_ERR_ARG;
    if (k->d > MFGP_MAX_D) return MFGP_UNSUPPORTED;
    int terms = 0;
    for (const mfgp_kernel* q = k; q; q = q->next) {
        if (++terms > MFGP_MAX_TERMS) return MFGP_UNSUPPORTED;
        const int st = check_term(q, k->d);
        if (st != MFGP_OK) return st;
    }
    if (!std::isfinite(k->noise) || k->noise < 0.0f) return MFGP_ERR_ARG;
    if (need_noise && !(k->noise > 0.0f)) return MFGP_ERR_ARG;
    return MFGP_OK;
}

// A product with a Matern or Linear factor: the general product of prod.hip,
// evaluated by the FP32 VALU sweeps only.
static bool general_product(const mfgp_kernel* k) {
    if (!k->times) return false;
    for (const mfgp_kernel* q = k; q; q = q->times)
        if (q->family != MFGP_RBF && q->family != MFGP_PERIODIC) return true;
    return false;
}

static bool any_general_product(const mfgp_kernel* k) {
    for (const mfgp_kernel* q = k; q; q = q->next)
        if (general_product(q)) return true;
    return false;
}

// The preconditioned calls take one stationary or periodic term (or a product
// of RBF and periodic factors).
static int check_precond_kernel(const mfgp_kernel* k, bool need_noise) {
    const int st = check_kernel(k, need_noise);
    if (st != MFGP_OK) return st;
    if (k->next || k->family == MFGP_LINEAR || general_product(k)) return MFGP_UNSUPPORTED;
    return MFGP_OK;
}

// The bf16 product forms do not take general products.
static int check_kernel_precision(const mfgp_kernel* k, int precision) {
    if (!is_fp32_class(precision) && any_general_product(k)) return MFGP_UNSUPPORTED;
    return MFGP_OK;
}

static int check_opts(const mfgp_cg_opts* o) {
    if (!o) return MFGP_ERR_ARG;
    if (!std::isfinite(o->tol) || !(o->tol > 0.0)) return MFGP_ERR_ARG;
    if (o->max_iter < 0) return MFGP_ERR_ARG;
    if (o->precision < MFGP_FP32 || o->precision > MFGP_FP32_GRAM) return MFGP_ERR_ARG;
    if (!precision_supported(o->precision)) return MFGP_UNSUPPORTED;
    return MFGP_OK;
}

// The BF16-MFMA sweeps hold at most two 32-column tiles.
static int check_precision_cols(int precision, int t) {
    if ((precision == MFGP_BF16X1 || precision == MFGP_BF16X2 || precision == MFGP_BF16X3) && t > 65)
        return MFGP_UNSUPPORTED;
    return MFGP_OK;
}

// Default CG iteration cap: 2n (at least 64, at most 20000).  Exact CG ends in
// n steps; in FP32 a well-conditioned small system may need a few more.
static int default_max_iter(int64_t n, int max_iter) {
    if (max_iter > 0) return max_iter;
    int64_t m = 2 * n;
    if (m < 64) m = 64;
    if (m > 20000) m = 20000;
    return static_cast<int>(m);
}

static int hip_fail(hipError_t e) {
    set_last_hip_error(e);
    return MFGP_ERR_HIP;
}

#define ABI_CHECK(expr)                    \
    do {                                   \
        hipError_t e_ = (expr);            \
        if (e_ != hipSuccess) return hip_fail(e_); \
    } while (0)

// ---------------------------------------------------------------- carving (shared by size queries)

struct MatvecWs { float* U; void* scratch; void* sum; };
static MatvecWs carve_matvec(Carver& cv, int64_t n, int d, int t, int precision) {
    MatvecWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    if (is_fp32_class(precision))
        w.scratch = cv.take<char>(apply_fp32_scratch_bytes(n, n, t, precision));
    else
        w.scratch = cv.take<char>(mfma_scratch_bytes(n, n, t, precision));
    w.sum = cv.take<char>(sum_scratch_bytes(n, t));
    return w;
}

struct ResidWs { float* U; double* scratch; double* dots; double* tmp; void* sum; };
static ResidWs carve_resid(Carver& cv, int64_t n, int d, int t) {
    ResidWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.scratch = cv.take<double>(resid_scratch_doubles(n, t));
    w.sum = cv.take<char>(sum_scratch_bytes(n, t));
    w.dots = cv.take<double>(dots_scratch_doubles(n, t));
    w.tmp = cv.take<double>(2 * static_cast<size_t>(t));
    return w;
}

struct CgWs { float* U; CgBufs b; };
static CgWs carve_cgws(Carver& cv, int64_t n, int d, int t, int precision) {
    CgWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.b = carve_cg(cv, n, t, precision);
    return w;
}

struct PredictWs { float* U; float* Us; void* scratch; void* sum; };
static PredictWs carve_predict(Carver& cv, int64_t n, int d, int64_t m, int t) {
    PredictWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.Us = cv.take<float>(static_cast<size_t>(m) * d);
    w.scratch = cv.take<char>(apply_fp32_scratch_bytes(m, n, t, MFGP_FP32));
    w.sum = cv.take<char>(sum_scratch_bytes(m, t));
    return w;
}

struct AdjWs { float* U; double* scratch; double* dots; double* tmp; void* sum; };
static AdjWs carve_adjoint(Carver& cv, int64_t n, int d, int t) {
    AdjWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.scratch = cv.take<double>(adjoint_scratch_doubles(n, d, t));
    w.sum = cv.take<char>(sum_scratch_bytes(n, t));
    w.dots = cv.take<double>(dots_scratch_doubles(n, t));
    w.tmp = cv.take<double>(2 * static_cast<size_t>(t) + 8);
    return w;
}

struct MllWs {
    float* U; float* Bm; double* X64; float* Zgen; double* coeff; double* tmp; CgBufs b;
    double* adj;
};
static MllWs carve_mll(Carver& cv, int64_t n, int d, int t, int precision, int max_iter) {
    MllWs w;
    const size_t nt = static_cast<size_t>(n) * t;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.Bm = cv.take<float>(nt);
    w.X64 = cv.take<double>(nt);
    w.Zgen = cv.take<float>(static_cast<size_t>(n) * (t - 1));
    w.coeff = cv.take<double>(static_cast<size_t>(t) * max_iter * 2);
    w.tmp = cv.take<double>(4 * static_cast<size_t>(t) + 8);
    w.b = carve_cg(cv, n, t, precision);
    w.adj = cv.take<double>(adjoint_scratch_doubles(n, d, t));
    return w;
}

// Preconditioned operations (rank-k pivoted Cholesky, Woodbury apply, PCG, MLL).
struct PcholWs { float* U; double* scratch; };
static PcholWs carve_pchol(Carver& cv, int64_t n, int d) {
    PcholWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.scratch = cv.take<double>(pchol_scratch_doubles(n));
    return w;
}
struct PapplyWs { double* pc; };
static PapplyWs carve_papply(Carver& cv, int64_t n, int k, int t) {
    PapplyWs w;
    w.pc = cv.take<double>(pc_scratch_doubles(n, k, t));
    return w;
}
struct PcgWs { float* U; CgBufs b; PcgBufs pb; };
static PcgWs carve_pcgws(Carver& cv, int64_t n, int d, int k, int t, int precision) {
    PcgWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.b = carve_cg(cv, n, t, precision);
    w.pb = carve_pcg(cv, n, k, t);
    return w;
}
struct PmllWs { MllWs m; PcgBufs pb; };
static PmllWs carve_pmll(Carver& cv, int64_t n, int d, int k, int t, int precision, int max_iter) {
    PmllWs w;
    w.m = carve_mll(cv, n, d, t, precision, max_iter);
    w.pb = carve_pcg(cv, n, k, t);
    return w;
}

// Index of d/d sigma^2 in the gradient: after every term's parameters.
static int noise_index(const mfgp_kernel* k) {
    int n = 0;
    for (const mfgp_kernel* q = k; q; q = q->next) n += term_params(*q);
    return n;
}

// Feature dimension of the prescaled coordinates (the d of the size queries).
static int feature_dim(const mfgp_kernel* k) { return chain_feature_dim(*k); }

static int check_matvec_args(const mfgp_kernel* kern, const float* X, int64_t n, const float* V, int t,
                             const float* KV, int precision) {
    int st = check_kernel(kern, false);
    if (st != MFGP_OK) return st;
    if (!X || !V || !KV || n < 1 || t < 1 || KV == V) return MFGP_ERR_ARG;
    if (precision < MFGP_FP32 || precision > MFGP_FP32_GRAM) return MFGP_ERR_ARG;
    if (!precision_supported(precision)) return MFGP_UNSUPPORTED;
    if ((st = check_kernel_precision(kern, precision)) != MFGP_OK) return st;
    return check_precision_cols(precision, t);
}

// The product on a workspace of at least mfgp_workspace_bytes(MFGP_OP_MATVEC)
// bytes; every scratch value is written by a kernel of this call before it is
// read, so the workspace needs no clearing between calls.
static int matvec_into(const mfgp_kernel* kern, const float* X, int64_t n, const float* V, int t, float* KV,
                       int precision, void* ws, hipStream_t s) {
    Carver cv(ws);
    MatvecWs w = carve_matvec(cv, n, feature_dim(kern), t, precision);
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    ABI_CHECK(apply_sum(op, nullptr, n, V, t, KV, true, V, w.scratch, w.sum, precision, s));
    return MFGP_OK;
}

// Workspace of mfgp_kernel_matvec_noalloc: a fixed device array, one copy per
// GPU for the life of the process.  In host code `scratch` names a host-side
// stand-in, never the device memory: its device address is looked up once per
// device (hipGetSymbolAddress with that device current) and only that address
// reaches the kernels.
constexpr size_t kNoAllocBytes = MFGP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the stream's device, which must be the
// current device (the lookup is made with it current).
static int noalloc_scratch(hipStream_t s, void** out) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e);
    hipDevice_t sdev = cur;
    if (s) {
        e = hipStreamGetDevice(s, &sdev);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (sdev != cur) return MFGP_ERR_ARG;
    if (cur < 0 || cur >= kMaxDevices) return MFGP_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[cur]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!p) return hip_fail(hipErrorInvalidSymbol);
        g_scratch_addr[cur] = p;
    }
    *out = g_scratch_addr[cur];
    return MFGP_OK;
}

}  // namespace mfgp

using namespace mfgp;

extern "C" {

int mfgp_version(void) { return 100; }

int mfgp_last_hip_error(void) { return g_last_hip; }

int mfgp_release_thread_resources(void) {
    hipError_t e = release_fft_plans();
    const hipError_t e2 = release_blas_handles();
    const hipError_t e3 = release_cg_streams();
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = e3;
    return e == hipSuccess ? MFGP_OK : hip_fail(e);
}

const char* mfgp_status_string(int status) {
    switch (status) {
        case MFGP_OK: return "ok";
        case MFGP_ERR_ARG: return "invalid argument";
        case MFGP_ERR_HIP: return "HIP runtime error";
        case MFGP_ERR_WORKSPACE: return "workspace too small";
        case MFGP_NOT_CONVERGED: return "not converged";
        case MFGP_BREAKDOWN: return "CG breakdown";
        case MFGP_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

int mfgp_num_params(const mfgp_kernel* k) {
    if (!k || k->d < 1) return 0;
    return noise_index(k) + 1;
}

int mfgp_feature_dim(const mfgp_kernel* k) {
    if (!k || k->d < 1) return 0;
    return feature_dim(k);
}

size_t mfgp_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t t, int32_t precision,
                            int32_t max_iter) {
    if (n < 1 || d < 1 || d > MFGP_MAX_TERMS * MFGP_MAX_D || t < 1) return 0;
    if (precision < MFGP_FP32 || precision > MFGP_FP32_GRAM) return 0;
    Carver cv(nullptr);
    switch (op) {
        case MFGP_OP_MATVEC: carve_matvec(cv, n, d, t, precision); break;
        case MFGP_OP_RESIDUAL: carve_resid(cv, n, d, t); break;
        case MFGP_OP_CG: carve_cgws(cv, n, d, t, precision); break;
        case MFGP_OP_PREDICT:
            if (max_iter < 1) return 0;
            carve_predict(cv, n, d, max_iter, t);
            break;
        case MFGP_OP_ADJOINT: carve_adjoint(cv, n, d, t); break;
        case MFGP_OP_MLL:
            if (t < 2) return 0;
            carve_mll(cv, n, d, t, precision, default_max_iter(n, max_iter));
            break;
        default: return 0;
    }
    return cv.off + 256;
}

int mfgp_kernel_matvec(const mfgp_kernel* kern, const float* X, int64_t n, const float* V,
                       int32_t t, float* KV, int32_t precision, void* ws, size_t ws_bytes,
                       void* stream) {
    int st = check_matvec_args(kern, X, n, V, t, KV, precision);
    if (st != MFGP_OK) return st;
    if (!ws) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_workspace_bytes(MFGP_OP_MATVEC, n, feature_dim(kern), t, precision, 0))
        return MFGP_ERR_WORKSPACE;
    return matvec_into(kern, X, n, V, t, KV, precision, ws, static_cast<hipStream_t>(stream));
}

int mfgp_kernel_matvec_noalloc(const mfgp_kernel* kern, const float* X, int64_t n, const float* V,
                               int32_t t, float* KV, int32_t precision, void* stream) {
    int st = check_matvec_args(kern, X, n, V, t, KV, precision);
    if (st != MFGP_OK) return st;
    if (mfgp_workspace_bytes(MFGP_OP_MATVEC, n, feature_dim(kern), t, precision, 0) > kNoAllocBytes)
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if ((st = noalloc_scratch(s, &ws)) != MFGP_OK) return st;
    return matvec_into(kern, X, n, V, t, KV, precision, ws, s);
}

int mfgp_residual(const mfgp_kernel* kern, const float* X, int64_t n, const float* B,
                  const double* Xsol, int32_t t, double* R, double* rel, void* ws,
                  size_t ws_bytes, void* stream) {
    int st = check_kernel(kern, false);
    if (st != MFGP_OK) return st;
    if (!X || !B || !Xsol || !R || !ws || n < 1 || t < 1) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_workspace_bytes(MFGP_OP_RESIDUAL, n, feature_dim(kern), t, 0, 0))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    ResidWs w = carve_resid(cv, n, feature_dim(kern), t);
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    ABI_CHECK(residual_sum(op, B, Xsol, t, R, w.scratch, w.sum, s));
    if (rel) {
        ABI_CHECK(col_dots_dd(R, R, n, t, w.tmp, w.dots, s));
        ABI_CHECK(col_dots_ff(B, B, n, t, w.tmp + t, w.dots, s));
        std::vector<double> h(2 * t);
        ABI_CHECK(hipMemcpyAsync(h.data(), w.tmp, 2 * t * sizeof(double), hipMemcpyDeviceToHost, s));
        ABI_CHECK(hipStreamSynchronize(s));
        for (int c = 0; c < t; ++c) rel[c] = h[t + c] > 0.0 ? std::sqrt(h[c] / h[t + c]) : 0.0;
    }
    return MFGP_OK;
}

int mfgp_cg_solve(const mfgp_kernel* kern, const float* X, int64_t n, const float* B, int32_t t,
                  double* Xsol, const mfgp_cg_opts* opts, mfgp_cg_info* info, double* lanczos,
                  void* ws, size_t ws_bytes, void* stream) {
    int st = check_kernel(kern, true);
    if (st != MFGP_OK) return st;
    if ((st = check_opts(opts)) != MFGP_OK) return st;
    if ((st = check_kernel_precision(kern, opts->precision)) != MFGP_OK) return st;
    if (!X || !B || !Xsol || !ws || n < 1 || t < 1) return MFGP_ERR_ARG;
    if ((st = check_precision_cols(opts->precision, t)) != MFGP_OK) return st;
    if (ws_bytes < mfgp_workspace_bytes(MFGP_OP_CG, n, feature_dim(kern), t, opts->precision, opts->max_iter))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    CgWs w = carve_cgws(cv, n, feature_dim(kern), t, opts->precision);
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    const int max_iter = default_max_iter(n, opts->max_iter);
    return cg_run(op, B, t, Xsol, *opts, info, lanczos, max_iter, w.b, s);
}

int mfgp_predict_mean(const mfgp_kernel* kern, const float* X, int64_t n, const float* Xs,
                      int64_t m, const float* A, int32_t t, float* MU, void* ws, size_t ws_bytes,
                      void* stream) {
    int st = check_kernel(kern, false);
    if (st != MFGP_OK) return st;
    if (!X || !Xs || !A || !MU || !ws || n < 1 || m < 1 || t < 1) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_workspace_bytes(MFGP_OP_PREDICT, n, feature_dim(kern), t, 0, static_cast<int32_t>(m)))
        return MFGP_ERR_WORKSPACE;
    if (m > 0x7fffffff) return MFGP_UNSUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    PredictWs w = carve_predict(cv, n, feature_dim(kern), m, t);
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    OpChain chs;
    make_chain(chs, *kern, Xs, m, w.Us);
    ABI_CHECK(prescale_chain(chs, s));
    ABI_CHECK(apply_sum(op, &chs.head(), m, A, t, MU, false, nullptr, w.scratch, w.sum, MFGP_FP32, s));
    return MFGP_OK;
}

struct VarWs { float* U; float* Us; float* Z; float* W; double* X64; float* U32; float* Q; CgBufs b; void* scratch; void* sum; };
static VarWs carve_variance(Carver& cv, int64_t n, int d, int64_t m, int p, int precision) {
    VarWs w;
    w.U = cv.take<float>(static_cast<size_t>(n) * d);
    w.Us = cv.take<float>(static_cast<size_t>(m) * d);
    w.Z = cv.take<float>(static_cast<size_t>(m) * p);
    w.W = cv.take<float>(static_cast<size_t>(n) * p);
    w.X64 = cv.take<double>(static_cast<size_t>(n) * p);
    w.U32 = cv.take<float>(static_cast<size_t>(n) * p);
    w.Q = cv.take<float>(static_cast<size_t>(m) * p);
    w.b = carve_cg(cv, n, p, precision);
    w.scratch = cv.take<char>(std::max(apply_fp32_scratch_bytes(n, m, p, MFGP_FP32),
                                       apply_fp32_scratch_bytes(m, n, p, MFGP_FP32)));
    w.sum = cv.take<char>(sum_scratch_bytes(std::max(n, m), p));
    return w;
}

size_t mfgp_variance_workspace_bytes(int64_t n, int32_t d, int64_t m, int32_t p, int32_t precision) {
    if (n < 1 || m < 1 || p < 1 || d < 1 || d > MFGP_MAX_TERMS * MFGP_MAX_D) return 0;
    if (precision < MFGP_FP32 || precision > MFGP_FP32_GRAM) return 0;
    Carver cv(nullptr);
    carve_variance(cv, n, d, m, p, precision);
    return cv.off + 256;
}

int mfgp_predict_variance(const mfgp_kernel* kern, const float* X, int64_t n, const float* Xs, int64_t m,
                          int32_t p, const float* Z, const mfgp_cg_opts* opts, float* var, mfgp_cg_info* info,
                          void* ws, size_t ws_bytes, void* stream) {
    int st = check_kernel(kern, true);
    if (st != MFGP_OK) return st;
    if ((st = check_opts(opts)) != MFGP_OK) return st;
    if ((st = check_kernel_precision(kern, opts->precision)) != MFGP_OK) return st;
    if (!X || !Xs || !var || !ws || n < 1 || m < 1 || p < 1) return MFGP_ERR_ARG;
    if ((st = check_precision_cols(opts->precision, p)) != MFGP_OK) return st;
    if (m > 0x7fffffff) return MFGP_UNSUPPORTED;
    if (ws_bytes < mfgp_variance_workspace_bytes(n, feature_dim(kern), m, p, opts->precision)) return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    VarWs w = carve_variance(cv, n, feature_dim(kern), m, p, opts->precision);
    OpChain ch, chs;
    make_chain(ch, *kern, X, n, w.U);
    make_chain(chs, *kern, Xs, m, w.Us);
    const Operator& op = ch.head();
    const Operator& ops = chs.head();
    ABI_CHECK(prescale_chain(ch, s));
    ABI_CHECK(prescale_chain(chs, s));
    const float* Zp = Z;
    if (!Zp) {
        ABI_CHECK(launch_rademacher(opts->probe_seed, m, p, w.Z, s));
        Zp = w.Z;
    }
    // W = K(X, Xs) Z (rows: training points, columns: test points)
    ABI_CHECK(apply_sum(ops, &op, n, Zp, p, w.W, false, nullptr, w.scratch, w.sum, MFGP_FP32, s));
    const int max_iter = default_max_iter(n, opts->max_iter);
    const int cst = cg_run(op, w.W, p, w.X64, *opts, info, nullptr, max_iter, w.b, s);
    if (cst == MFGP_ERR_HIP) return cst;
    ABI_CHECK(f64_to_f32(w.X64, w.U32, n * p, s));
    // Q = K(Xs, X) K_y^{-1} W
    ABI_CHECK(apply_sum(op, &ops, m, w.U32, p, w.Q, false, nullptr, w.scratch, w.sum, MFGP_FP32, s));
    ABI_CHECK(diag_variance(Zp, w.Q, m, p, stationary_prior(op), var, s));
    ABI_CHECK(add_linear_prior(ops, m, var, s));
    ABI_CHECK(hipStreamSynchronize(s));
    return cst;
}

int mfgp_slq_quadrature(const double* coeffs, int32_t m, double znorm2, double* q) {
    if (!coeffs || !q || m < 1 || !(znorm2 >= 0.0)) return MFGP_ERR_ARG;
    return slq_quadrature(coeffs, m, znorm2, q);
}

int mfgp_rademacher(uint64_t seed, int64_t n, int32_t p, float* Z, void* stream) {
    if (!Z || n < 1 || p < 1) return MFGP_ERR_ARG;
    ABI_CHECK(launch_rademacher(seed, n, p, Z, static_cast<hipStream_t>(stream)));
    return MFGP_OK;
}

int mfgp_kernel_adjoint(const mfgp_kernel* kern, const float* X, int64_t n, const float* A,
                        const float* B, int32_t t, const double* colw, double* grad, void* ws,
                        size_t ws_bytes, void* stream) {
    int st = check_kernel(kern, false);
    if (st != MFGP_OK) return st;
    if (!X || !A || !B || !colw || !grad || !ws || n < 1 || t < 1) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_workspace_bytes(MFGP_OP_ADJOINT, n, feature_dim(kern), t, 0, 0))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    AdjWs w = carve_adjoint(cv, n, feature_dim(kern), t);
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    ABI_CHECK(chain_gradient(op, A, B, t, colw, grad, w.scratch, w.sum, s));
    ABI_CHECK(col_dots_ff(A, B, n, t, w.tmp, w.dots, s));
    std::vector<double> ab(t);
    ABI_CHECK(hipMemcpyAsync(ab.data(), w.tmp, t * sizeof(double), hipMemcpyDeviceToHost, s));
    ABI_CHECK(hipStreamSynchronize(s));
    double sn = 0.0;
    for (int c = 0; c < t; ++c) sn += colw[c] * ab[c];
    grad[noise_index(kern)] = sn;
    return MFGP_OK;
}

}  // extern "C"

// The quadratures e_1^T log(T_c) e_1 ||z_c||^2 of columns 1..t-1 (column 0 is
// the data column) from their CG coefficients cf[c] (len[c] pairs), on up to
// min(cores, t - 1) host threads; a thread the system refuses to start
// leaves its share to the calling thread, so no exception leaves the library.
static void run_quadratures(int t, const std::vector<int>& len, const std::vector<std::vector<double>>& cf,
                            const double* znorm2, std::vector<double>& q, std::vector<int>& qs) {
    const int p = t - 1;
    q.assign(t, 0.0);
    qs.assign(t, MFGP_OK);
    if (p < 1) return;
    const unsigned hw = std::thread::hardware_concurrency();
    const int nth = static_cast<int>(std::min<unsigned>(hw ? hw : 1, static_cast<unsigned>(p)));
    auto work = [&](int th) {
        for (int c = 1 + th; c < t; c += nth)
            qs[c] = len[c] < 1 ? MFGP_BREAKDOWN : slq_quadrature(cf[c].data(), len[c], znorm2[c], &q[c]);
    };
    std::vector<std::thread> pool;
    int started = 0;
    for (; started < nth; ++started) {
        try {
            pool.emplace_back(work, started);
        } catch (...) {
            break;
        }
    }
    for (int th = started; th < nth; ++th) work(th);
    for (auto& th : pool) th.join();
}

// log|K_y| ~ (1/p) sum over the probe columns c = 1 .. t-1 of ||z_c||^2
// e_1^T log(T_c) e_1 (stochastic Lanczos quadrature, Sec. 3 "Inference"),
// T_c from the CG coefficients in coeff [t][max_iter][2] (device); bnorm2
// (host, [t]) holds ||z_c||^2.  The quadratures run in parallel host threads.
// *slq_status is MFGP_BREAKDOWN if a probe's quadrature failed.
static hipError_t probe_logdet(const std::vector<mfgp_cg_info>& inf, const double* coeff, int max_iter,
                               const double* bnorm2, int t, double* ld, int* slq_status, hipStream_t s) {
    const int p = t - 1;
    std::vector<std::vector<double>> cf(t);
    for (int c = 1; c < t; ++c) {
        cf[c].resize(2 * static_cast<size_t>(inf[c].lanczos_len > 0 ? inf[c].lanczos_len : 1));
        if (inf[c].lanczos_len > 0) {
            hipError_t e = hipMemcpyAsync(cf[c].data(), coeff + static_cast<size_t>(c) * max_iter * 2,
                                          2 * inf[c].lanczos_len * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    std::vector<int> len(t, 0);
    for (int c = 1; c < t; ++c) len[c] = inf[c].lanczos_len;
    std::vector<double> q;
    std::vector<int> qs;
    run_quadratures(t, len, cf, bnorm2, q, qs);
    double sum = 0.0;
    *slq_status = MFGP_OK;
    for (int c = 1; c < t; ++c) {
        sum += q[c];
        if (qs[c] != MFGP_OK) *slq_status = MFGP_BREAKDOWN;
    }
    *ld = sum / p;
    return hipSuccess;
}

extern "C" {

int mfgp_mll_and_grad(const mfgp_kernel* kern, const float* X, int64_t n, const float* y,
                      int32_t num_probes, const float* Z, const mfgp_cg_opts* opts, double* mll,
                      double* logdet, double* grad, double* alpha_out, mfgp_cg_info* info,
                      void* ws, size_t ws_bytes, void* stream) {
    int st = check_kernel(kern, true);
    if (st != MFGP_OK) return st;
    if ((st = check_opts(opts)) != MFGP_OK) return st;
    if ((st = check_kernel_precision(kern, opts->precision)) != MFGP_OK) return st;
    if (!X || !y || !mll || !ws || n < 1 || num_probes < 1) return MFGP_ERR_ARG;
    const int p = num_probes;
    const int t = p + 1;
    if ((st = check_precision_cols(opts->precision, t)) != MFGP_OK) return st;
    const int max_iter = default_max_iter(n, opts->max_iter);
    if (ws_bytes < mfgp_workspace_bytes(MFGP_OP_MLL, n, feature_dim(kern), t, opts->precision, max_iter))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    MllWs w = carve_mll(cv, n, feature_dim(kern), t, opts->precision, max_iter);
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    const float* Zp = Z;
    if (!Zp) {
        ABI_CHECK(launch_rademacher(opts->probe_seed, n, p, w.Zgen, s));
        Zp = w.Zgen;
    }
    hipLaunchKernelGGL(pack_yz_kernel, dim3(nb(n * t)), dim3(256), 0, s, y, Zp, n, p, w.Bm);
    ABI_CHECK(hipGetLastError());

    using clock = std::chrono::steady_clock;
    auto ms_since = [](clock::time_point a) {
        return std::chrono::duration<double, std::milli>(clock::now() - a).count();
    };
    if (timing_on()) ABI_CHECK(hipStreamSynchronize(s));
    auto t0 = clock::now();
    std::vector<mfgp_cg_info> inf(t);
    mfgp_cg_opts o = *opts;
    o.warm_start = 0;
    const int cg_status = cg_run(op, w.Bm, t, w.X64, o, inf.data(), w.coeff, max_iter, w.b, s);
    timing_phase(0, ms_since(t0));
    t0 = clock::now();
    if (cg_status == MFGP_ERR_HIP || cg_status == MFGP_ERR_ARG) return cg_status;
    if (info) std::memcpy(info, inf.data(), t * sizeof(mfgp_cg_info));

    // Column dot products in FP64: b_c^T b_c, x_c^T b_c, x_c^T x_c.
    double* bb = w.tmp;
    double* xb = w.tmp + t;
    double* xx = w.tmp + 2 * t;
    ABI_CHECK(col_dots_ff(w.Bm, w.Bm, n, t, bb, w.b.dots, s));
    ABI_CHECK(col_dots_df(w.X64, w.Bm, n, t, xb, w.b.dots, s));
    ABI_CHECK(col_dots_dd(w.X64, w.X64, n, t, xx, w.b.dots, s));
    std::vector<double> h(3 * t);
    ABI_CHECK(hipMemcpyAsync(h.data(), w.tmp, 3 * t * sizeof(double), hipMemcpyDeviceToHost, s));
    if (alpha_out) {
        hipLaunchKernelGGL(copy_col0_kernel, dim3(nb(n)), dim3(256), 0, s, w.X64, alpha_out, n, t);
        ABI_CHECK(hipGetLastError());
    }
    double ld = 0.0;
    int slq_status = MFGP_OK;
    ABI_CHECK(probe_logdet(inf, w.coeff, max_iter, h.data(), t, &ld, &slq_status, s));
    timing_phase(1, ms_since(t0));
    t0 = clock::now();
    const double two_pi = 6.283185307179586477;
    *mll = -0.5 * (h[t + 0] + ld + static_cast<double>(n) * std::log(two_pi));
    if (logdet) *logdet = ld;

    if (grad) {
        // A = fl32([alpha, U]) into R, B = [fl32(alpha), Z] into P (CG buffers are free now).
        float* Ag = w.b.R;
        float* Bg = w.b.P;
        ABI_CHECK(f64_to_f32(w.X64, Ag, n * t, s));
        ABI_CHECK(copy2_f32(w.Bm, Bg, Bg, n * t, s));
        hipLaunchKernelGGL(set_col0_kernel, dim3(nb(n)), dim3(256), 0, s, w.X64, Bg, n, t);
        ABI_CHECK(hipGetLastError());
        std::vector<double> colw(t, -0.5 / p);
        colw[0] = 0.5;
        ABI_CHECK(chain_gradient(op, Ag, Bg, t, colw.data(), grad, w.adj, w.b.sum, s));
        double tr = 0.0;
        for (int c = 1; c < t; ++c) tr += h[t + c];
        grad[noise_index(kern)] = 0.5 * h[2 * t + 0] - 0.5 * tr / p;
        timing_phase(2, ms_since(t0));
    }
    if (cg_status != MFGP_OK) return cg_status;
    return slq_status;
}

// ---------------------------------------------------------------- structured kernel interpolation

static int check_ski(const mfgp_kernel* kern, const mfgp_ski_grid* grid, bool need_noise) {
    int st = check_kernel(kern, need_noise);
    if (st != MFGP_OK) return st;
    if (!grid) return MFGP_ERR_ARG;
    if (kern->next || kern->times || kern->family == MFGP_LINEAR || kern->d > 3) return MFGP_UNSUPPORTED;
    int64_t lr = 1;
    for (int k = 0; k < kern->d; ++k) {
        if (grid->m[k] < 5) return MFGP_ERR_ARG;
        lr *= 2 * static_cast<int64_t>(grid->m[k]);
        if (lr >= (int64_t(1) << 31)) return MFGP_UNSUPPORTED;
        if (grid->explicit_range &&
            !(std::isfinite(grid->lo[k]) && std::isfinite(grid->hi[k]) && grid->hi[k] >= grid->lo[k]))
            return MFGP_ERR_ARG;
    }
    return MFGP_OK;
}

struct SkiMllWs { void* sk; void* gs; CgBufs b; float* Bm; double* X64; float* Zgen; double* coeff; double* tmp; };
static SkiMllWs carve_ski_mll(Carver& cv, int64_t n, int d, const int32_t* m, int t, int max_iter) {
    SkiMllWs w;
    const size_t nt = static_cast<size_t>(n) * t;
    w.sk = cv.take<char>(ski_scratch_bytes(d, m, t, n));
    w.gs = cv.take<char>(ski_grad_scratch_bytes(d, m, t));
    w.b = carve_cg_vectors(cv, n, t);
    w.Bm = cv.take<float>(nt);
    w.X64 = cv.take<double>(nt);
    w.Zgen = cv.take<float>(static_cast<size_t>(n) * (t - 1));
    w.coeff = cv.take<double>(static_cast<size_t>(t) * max_iter * 2);
    w.tmp = cv.take<double>(4 * static_cast<size_t>(t) + 8);
    return w;
}

size_t mfgp_ski_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t t, const mfgp_ski_grid* grid) {
    if (n < 1 || d < 1 || d > 3 || t < 1 || !grid) return 0;
    for (int k = 0; k < d; ++k)
        if (grid->m[k] < 5) return 0;
    Carver cv(nullptr);
    if (op == MFGP_OP_MLL) {
        // t = probes + 1; the CG iteration cap as mfgp_ski_mll_and_grad takes it (default)
        if (t < 2) return 0;
        carve_ski_mll(cv, n, d, grid->m, t, default_max_iter(n, 0));
        return cv.off + 256;
    }
    cv.take<char>(ski_scratch_bytes(d, grid->m, t, n));
    if (op == MFGP_OP_CG)
        carve_cg_vectors(cv, n, t);
    else if (op != MFGP_OP_MATVEC && op != MFGP_OP_PREDICT)
        return 0;
    return cv.off + 256;
}

int mfgp_ski_matvec(const mfgp_kernel* kern, const float* X, int64_t n, const mfgp_ski_grid* grid,
                    const float* V, int32_t t, float* KV, void* ws, size_t ws_bytes, void* stream) {
    int st = check_ski(kern, grid, false);
    if (st != MFGP_OK) return st;
    if (!X || !V || !KV || !ws || n < 1 || t < 1 || t > MFGP_MAX_T || KV == V) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_ski_workspace_bytes(MFGP_OP_MATVEC, n, kern->d, t, grid)) return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    void* sk_scratch = cv.take<char>(ski_scratch_bytes(kern->d, grid->m, t, n));
    SkiOp sk;
    const bool ex = grid->explicit_range != 0;
    ABI_CHECK(ski_setup(sk, *kern, X, n, nullptr, 0, grid->m, ex ? grid->lo : nullptr, ex ? grid->hi : nullptr, t,
                        sk_scratch, s));
    ABI_CHECK(ski_apply(sk, X, n, X, n, V, t, KV, true, kern->noise, V, s));
    return MFGP_OK;
}

int mfgp_ski_cg_solve(const mfgp_kernel* kern, const float* X, int64_t n, const mfgp_ski_grid* grid,
                      const float* B, int32_t t, double* Xsol, const mfgp_cg_opts* opts, mfgp_cg_info* info,
                      void* ws, size_t ws_bytes, void* stream) {
    int st = check_ski(kern, grid, true);
    if (st != MFGP_OK) return st;
    if ((st = check_opts(opts)) != MFGP_OK) return st;
    if (!X || !B || !Xsol || !ws || n < 1 || t < 1 || t > MFGP_MAX_T) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_ski_workspace_bytes(MFGP_OP_CG, n, kern->d, t, grid)) return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    void* sk_scratch = cv.take<char>(ski_scratch_bytes(kern->d, grid->m, t, n));
    CgBufs b = carve_cg_vectors(cv, n, t);
    SkiOp sk;
    const bool ex = grid->explicit_range != 0;
    ABI_CHECK(ski_setup(sk, *kern, X, n, nullptr, 0, grid->m, ex ? grid->lo : nullptr, ex ? grid->hi : nullptr, t,
                        sk_scratch, s));
    Operator op;
    op.family = kern->family;
    op.d = op.din = kern->d;
    op.n = n;
    op.s2 = kern->outputscale;
    op.sig2 = kern->noise;
    op.X = X;
    op.ski = &sk;
    const int max_iter = default_max_iter(n, opts->max_iter);
    return cg_run(op, B, t, Xsol, *opts, info, nullptr, max_iter, b, s);
}

int mfgp_ski_predict_mean(const mfgp_kernel* kern, const float* X, int64_t n, const float* Xs, int64_t m,
                          const mfgp_ski_grid* grid, const float* A, int32_t t, float* MU, void* ws,
                          size_t ws_bytes, void* stream) {
    int st = check_ski(kern, grid, false);
    if (st != MFGP_OK) return st;
    if (!X || !Xs || !A || !MU || !ws || n < 1 || m < 1 || t < 1 || t > MFGP_MAX_T) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_ski_workspace_bytes(MFGP_OP_PREDICT, n, kern->d, t, grid)) return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    void* sk_scratch = cv.take<char>(ski_scratch_bytes(kern->d, grid->m, t, n));
    SkiOp sk;
    const bool ex = grid->explicit_range != 0;
    ABI_CHECK(ski_setup(sk, *kern, X, n, Xs, m, grid->m, ex ? grid->lo : nullptr, ex ? grid->hi : nullptr, t,
                        sk_scratch, s));
    ABI_CHECK(ski_apply(sk, X, n, Xs, m, A, t, MU, false, 0.0f, nullptr, s));
    return MFGP_OK;
}

int mfgp_ski_mll_and_grad(const mfgp_kernel* kern, const float* X, int64_t n, const mfgp_ski_grid* grid,
                          const float* y, int32_t num_probes, const float* Z, const mfgp_cg_opts* opts, double* mll,
                          double* logdet, double* grad, mfgp_cg_info* info, void* ws, size_t ws_bytes,
                          void* stream) {
    int st = check_ski(kern, grid, true);
    if (st != MFGP_OK) return st;
    if ((st = check_opts(opts)) != MFGP_OK) return st;
    if (!X || !y || !mll || !ws || n < 1 || num_probes < 1 || num_probes + 1 > MFGP_MAX_T) return MFGP_ERR_ARG;
    if (opts->max_iter != 0) return MFGP_ERR_ARG;   // the workspace query assumes the default cap
    const int p = num_probes;
    const int t = p + 1;
    const int max_iter = default_max_iter(n, 0);
    if (ws_bytes < mfgp_ski_workspace_bytes(MFGP_OP_MLL, n, kern->d, t, grid)) return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    SkiMllWs w = carve_ski_mll(cv, n, kern->d, grid->m, t, max_iter);
    SkiOp sk;
    const bool ex = grid->explicit_range != 0;
    ABI_CHECK(ski_setup(sk, *kern, X, n, nullptr, 0, grid->m, ex ? grid->lo : nullptr, ex ? grid->hi : nullptr, t,
                        w.sk, s));
    Operator op;
    op.family = kern->family;
    op.d = op.din = kern->d;
    op.n = n;
    op.s2 = kern->outputscale;
    op.sig2 = kern->noise;
    op.X = X;
    op.ski = &sk;
    const float* Zp = Z;
    if (!Zp) {
        ABI_CHECK(launch_rademacher(opts->probe_seed, n, p, w.Zgen, s));
        Zp = w.Zgen;
    }
    hipLaunchKernelGGL(pack_yz_kernel, dim3(nb(n * t)), dim3(256), 0, s, y, Zp, n, p, w.Bm);
    ABI_CHECK(hipGetLastError());
    std::vector<mfgp_cg_info> inf(t);
    mfgp_cg_opts o = *opts;
    o.warm_start = 0;
    const int cg_status = cg_run(op, w.Bm, t, w.X64, o, inf.data(), w.coeff, max_iter, w.b, s);
    if (cg_status == MFGP_ERR_HIP || cg_status == MFGP_ERR_ARG) return cg_status;
    if (info) std::memcpy(info, inf.data(), t * sizeof(mfgp_cg_info));
    // b_c^T b_c, x_c^T b_c, x_c^T x_c in FP64
    double* bb = w.tmp;
    double* xb = w.tmp + t;
    double* xx = w.tmp + 2 * t;
    ABI_CHECK(col_dots_ff(w.Bm, w.Bm, n, t, bb, w.b.dots, s));
    ABI_CHECK(col_dots_df(w.X64, w.Bm, n, t, xb, w.b.dots, s));
    ABI_CHECK(col_dots_dd(w.X64, w.X64, n, t, xx, w.b.dots, s));
    std::vector<double> h(3 * t);
    ABI_CHECK(hipMemcpyAsync(h.data(), w.tmp, 3 * t * sizeof(double), hipMemcpyDeviceToHost, s));
    double ld = 0.0;
    int slq_status = MFGP_OK;
    ABI_CHECK(probe_logdet(inf, w.coeff, max_iter, h.data(), t, &ld, &slq_status, s));
    const double two_pi = 6.283185307179586477;
    *mll = -0.5 * (h[t + 0] + ld + static_cast<double>(n) * std::log(two_pi));
    if (logdet) *logdet = ld;
    if (grad) {
        // A = fl32([alpha, U]), B = [fl32(alpha), Z]; the CG vectors are free now
        float* Ag = w.b.R;
        float* Bg = w.b.P;
        ABI_CHECK(f64_to_f32(w.X64, Ag, n * t, s));
        ABI_CHECK(copy2_f32(w.Bm, Bg, Bg, n * t, s));
        hipLaunchKernelGGL(set_col0_kernel, dim3(nb(n)), dim3(256), 0, s, w.X64, Bg, n, t);
        ABI_CHECK(hipGetLastError());
        std::vector<double> colw(t, -0.5 / p);
        colw[0] = 0.5;
        ABI_CHECK(ski_gradient(sk, *kern, X, n, Ag, Bg, t, colw.data(), grad, w.gs, s));
        double tr = 0.0;
        for (int c = 1; c < t; ++c) tr += h[t + c];
        grad[noise_index(kern)] = 0.5 * h[2 * t + 0] - 0.5 * tr / p;
    }
    if (cg_status != MFGP_OK) return cg_status;
    return slq_status;
}

// ---------------------------------------------------------------- preconditioned solves

size_t mfgp_precond_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t t, int32_t rank,
                                    int32_t precision, int32_t max_iter) {
    if (n < 1 || d < 1 || d > MFGP_MAX_D || t < 1 || rank < 0 || rank > n || rank > MFGP_MAX_RANK) return 0;
    if (precision < MFGP_FP32 || precision > MFGP_FP32_GRAM) return 0;
    Carver cv(nullptr);
    switch (op) {
        case MFGP_OP_PCHOL: carve_pchol(cv, n, d); break;
        case MFGP_OP_PAPPLY: carve_papply(cv, n, rank, t); break;
        case MFGP_OP_PCG: carve_pcgws(cv, n, d, rank, t, precision); break;
        case MFGP_OP_PMLL:
            if (t < 2) return 0;
            carve_pmll(cv, n, d, rank, t, precision, default_max_iter(n, max_iter));
            break;
        default: return 0;
    }
    return cv.off + 256;
}

int mfgp_pivoted_cholesky(const mfgp_kernel* kern, const float* X, int64_t n, int32_t rank, float* L,
                          int32_t* piv, void* ws, size_t ws_bytes, void* stream) {
    int st = check_precond_kernel(kern, false);
    if (st != MFGP_OK) return st;
    if (!X || !L || !piv || !ws || n < 1 || rank < 1 || rank > n || rank > MFGP_MAX_RANK) return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_precond_workspace_bytes(MFGP_OP_PCHOL, n, feature_dim(kern), 1, rank, MFGP_FP32, 0))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    PcholWs w = carve_pchol(cv, n, feature_dim(kern));
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    ABI_CHECK(pivoted_cholesky(op, rank, L, piv, w.scratch, s));
    return MFGP_OK;
}

int mfgp_precond_probes(const float* L, int64_t n, int32_t rank, float noise, const float* E, const float* G,
                        int32_t p, float* Z, void* stream) {
    if (!G || !Z || n < 1 || p < 1 || rank < 0 || rank > n || (rank > 0 && (!L || !E)) ||
        !(std::isfinite(noise) && noise > 0.0f))
        return MFGP_ERR_ARG;
    ABI_CHECK(pc_probes(L, rank, n, noise, E, G, p, Z, static_cast<hipStream_t>(stream)));
    return MFGP_OK;
}

int mfgp_precond_apply(const float* L, int64_t n, int32_t rank, float noise, const float* R, int32_t t,
                       float* Zout, double* logdet, void* ws, size_t ws_bytes, void* stream) {
    if (!R || !Zout || !ws || n < 1 || t < 1 || rank < 0 || rank > n || rank > MFGP_MAX_RANK ||
        (rank > 0 && !L) || !(std::isfinite(noise) && noise > 0.0f))
        return MFGP_ERR_ARG;
    if (ws_bytes < mfgp_precond_workspace_bytes(MFGP_OP_PAPPLY, n, 1, t, rank, MFGP_FP32, 0))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    PapplyWs w = carve_papply(cv, n, rank, t);
    Precond pc;
    pc.L = L;
    pc.k = rank;
    pc.n = n;
    pc.s2n = noise;
    hipError_t e = pc_setup(pc, w.pc, s);
    if (e == hipErrorInvalidValue) return MFGP_BREAKDOWN;
    ABI_CHECK(e);
    if (logdet) *logdet = pc.logdet;
    ABI_CHECK(pc_apply(pc, R, t, Zout, w.pc, s));
    return MFGP_OK;
}

int mfgp_precond_cg_solve(const mfgp_kernel* kern, const float* X, int64_t n, const float* B, int32_t t,
                          double* Xsol, const float* L, int32_t rank, const mfgp_cg_opts* opts,
                          mfgp_cg_info* info, double* lanczos, void* ws, size_t ws_bytes, void* stream) {
    int st = check_precond_kernel(kern, true);
    if (st != MFGP_OK) return st;
    if ((st = check_opts(opts)) != MFGP_OK) return st;
    if (!X || !B || !Xsol || !ws || n < 1 || t < 1 || rank < 0 || rank > n || rank > MFGP_MAX_RANK ||
        (rank > 0 && !L))
        return MFGP_ERR_ARG;
    if ((st = check_precision_cols(opts->precision, t)) != MFGP_OK) return st;
    if (ws_bytes < mfgp_precond_workspace_bytes(MFGP_OP_PCG, n, feature_dim(kern), t, rank, opts->precision, opts->max_iter))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    PcgWs w = carve_pcgws(cv, n, feature_dim(kern), rank, t, opts->precision);
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    Precond pc;
    pc.L = L;
    pc.k = rank;
    pc.n = n;
    pc.s2n = kern->noise;
    hipError_t e = pc_setup(pc, w.pb.pc, s);
    if (e == hipErrorInvalidValue) return MFGP_BREAKDOWN;
    ABI_CHECK(e);
    const int max_iter = default_max_iter(n, opts->max_iter);
    return pcg_run(op, pc, B, t, Xsol, *opts, info, lanczos, max_iter, w.b, w.pb, s);
}

int mfgp_precond_mll_and_grad(const mfgp_kernel* kern, const float* X, int64_t n, const float* y,
                              int32_t num_probes, const float* Z, const float* L, int32_t rank,
                              const mfgp_cg_opts* opts, double* mll, double* logdet, double* grad,
                              double* alpha_out, mfgp_cg_info* info, void* ws, size_t ws_bytes, void* stream) {
    int st = check_precond_kernel(kern, true);
    if (st != MFGP_OK) return st;
    if ((st = check_opts(opts)) != MFGP_OK) return st;
    if (!X || !y || !Z || !mll || !ws || n < 1 || num_probes < 1 || rank < 0 || rank > n ||
        rank > MFGP_MAX_RANK || (rank > 0 && !L))
        return MFGP_ERR_ARG;
    const int p = num_probes;
    const int t = p + 1;
    if ((st = check_precision_cols(opts->precision, t)) != MFGP_OK) return st;
    const int max_iter = default_max_iter(n, opts->max_iter);
    if (ws_bytes < mfgp_precond_workspace_bytes(MFGP_OP_PMLL, n, feature_dim(kern), t, rank, opts->precision, max_iter))
        return MFGP_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    PmllWs W = carve_pmll(cv, n, feature_dim(kern), rank, t, opts->precision, max_iter);
    MllWs& w = W.m;
    OpChain ch;
    make_chain(ch, *kern, X, n, w.U);
    const Operator& op = ch.head();
    ABI_CHECK(prescale_chain(ch, s));
    hipLaunchKernelGGL(pack_yz_kernel, dim3(nb(n * t)), dim3(256), 0, s, y, Z, n, p, w.Bm);
    ABI_CHECK(hipGetLastError());
    Precond pc;
    pc.L = L;
    pc.k = rank;
    pc.n = n;
    pc.s2n = kern->noise;
    {
        hipError_t e = pc_setup(pc, W.pb.pc, s);
        if (e == hipErrorInvalidValue) return MFGP_BREAKDOWN;
        ABI_CHECK(e);
    }

    using clock = std::chrono::steady_clock;
    auto ms_since = [](clock::time_point a) {
        return std::chrono::duration<double, std::milli>(clock::now() - a).count();
    };
    if (timing_on()) ABI_CHECK(hipStreamSynchronize(s));
    auto t0 = clock::now();
    std::vector<mfgp_cg_info> inf(t);
    mfgp_cg_opts o = *opts;
    o.warm_start = 0;
    const int cg_status = pcg_run(op, pc, w.Bm, t, w.X64, o, inf.data(), w.coeff, max_iter, w.b, W.pb, s);
    timing_phase(0, ms_since(t0));
    t0 = clock::now();
    if (cg_status == MFGP_ERR_HIP || cg_status == MFGP_ERR_ARG) return cg_status;
    if (info) std::memcpy(info, inf.data(), t * sizeof(mfgp_cg_info));

    // FP64 column dots: x_c^T b_c and x_c^T x_c; b^T P^{-1} b of the probes.
    double* xb = w.tmp;
    double* xx = w.tmp + t;
    ABI_CHECK(col_dots_df(w.X64, w.Bm, n, t, xb, w.b.dots, s));
    ABI_CHECK(col_dots_dd(w.X64, w.X64, n, t, xx, w.b.dots, s));
    std::vector<double> h(2 * t), rz0(t);
    ABI_CHECK(hipMemcpyAsync(h.data(), w.tmp, 2 * t * sizeof(double), hipMemcpyDeviceToHost, s));
    ABI_CHECK(hipMemcpyAsync(rz0.data(), W.pb.rz0, t * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<std::vector<double>> cf(t);
    for (int c = 1; c < t; ++c) {
        cf[c].resize(2 * static_cast<size_t>(inf[c].lanczos_len > 0 ? inf[c].lanczos_len : 1));
        if (inf[c].lanczos_len > 0)
            ABI_CHECK(hipMemcpyAsync(cf[c].data(), w.coeff + static_cast<size_t>(c) * max_iter * 2,
                                     2 * inf[c].lanczos_len * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (alpha_out) {
        hipLaunchKernelGGL(copy_col0_kernel, dim3(nb(n)), dim3(256), 0, s, w.X64, alpha_out, n, t);
        ABI_CHECK(hipGetLastError());
    }
    ABI_CHECK(hipStreamSynchronize(s));

    // log|K_y| = log|P| + (1/p) sum_c (z_c^T P^{-1} z_c) e_1^T log(T_c) e_1.
    std::vector<int> len(t, 0);
    for (int c = 1; c < t; ++c) len[c] = inf[c].lanczos_len;
    std::vector<double> q;
    std::vector<int> qs;
    run_quadratures(t, len, cf, rz0.data(), q, qs);
    double ld = 0.0;
    int slq_status = MFGP_OK;
    for (int c = 1; c < t; ++c) {
        ld += q[c];
        if (qs[c] != MFGP_OK) slq_status = MFGP_BREAKDOWN;
    }
    ld = pc.logdet + ld / p;
    timing_phase(1, ms_since(t0));
    t0 = clock::now();
    const double two_pi = 6.283185307179586477;
    *mll = -0.5 * (h[0] + ld + static_cast<double>(n) * std::log(two_pi));
    if (logdet) *logdet = ld;

    if (grad) {
        // A = fl32([alpha, U]), B = [fl32(alpha), P^{-1} Z]: the trace term pairs
        // u_c = K_y^{-1} z_c with w_c = P^{-1} z_c.
        float* Ag = w.b.R;
        float* Bg = w.b.P;
        ABI_CHECK(f64_to_f32(w.X64, Ag, n * t, s));
        ABI_CHECK(pc_apply(pc, w.Bm, t, Bg, W.pb.pc, s));
        hipLaunchKernelGGL(set_col0_kernel, dim3(nb(n)), dim3(256), 0, s, w.X64, Bg, n, t);
        ABI_CHECK(hipGetLastError());
        std::vector<double> colw(t, -0.5 / p);
        colw[0] = 0.5;
        ABI_CHECK(chain_gradient(op, Ag, Bg, t, colw.data(), grad, w.adj, w.b.sum, s));
        // d/d sigma^2: dK_y = I, so 1/2 a^T a - 1/2 (1/p) sum_c u_c^T w_c (FP64 dots)
        double* uw = w.tmp;
        ABI_CHECK(col_dots_df(w.X64, Bg, n, t, uw, w.b.dots, s));
        std::vector<double> huw(t);
        ABI_CHECK(hipMemcpyAsync(huw.data(), uw, t * sizeof(double), hipMemcpyDeviceToHost, s));
        ABI_CHECK(hipStreamSynchronize(s));
        double tr = 0.0;
        for (int c = 1; c < t; ++c) tr += huw[c];
        grad[noise_index(kern)] = 0.5 * h[t + 0] - 0.5 * tr / p;
        timing_phase(2, ms_since(t0));
    }
    if (cg_status != MFGP_OK) return cg_status;
    return slq_status;
}

}  // extern "C"
