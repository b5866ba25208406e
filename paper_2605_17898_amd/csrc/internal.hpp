// Internal host-side interfaces between the C ABI and the kernels.
#pragma once

#include "common.hpp"

namespace mfgp {

// A kernel operator bound to its training inputs: family, prescale factors
// and the prescaled coordinates U (device, [n, d]) that the sweeps read.
// The periodic family is held as RBF on its d = 2 din circle features
// u = c (cos 2 pi x / p, sin 2 pi x / p) / l (periodic = 1, din the input
// dimension, period p); for the other families din = d.
// Structured kernel interpolation (ski.hip): the regular grid of D <= 3
// dimensions (m_k nodes, circulant embedding L_k = 2 m_k), the device grid
// geometry geo = [lo_0..2, h_0..2], the FP64 spectrum of the embedded grid
// kernel (lam, complex [Lc]) and the product buffers for t columns.
struct SkiGeomH {
    int d;
    int m[3];
    int L[3];
    int64_t Lr;   // prod L
    int64_t Lc;   // (L0 / 2 + 1) L1 L2
};
// The training points are bucketed once by the cell of their stencil
// (cells b_k in [-2, m_k], ncell of them): offsets [ncell + 1] into perm [n].
struct SkiOp {
    SkiGeomH g{};
    double* geo = nullptr;
    void* lam = nullptr;
    double* grid = nullptr;   // [t][Lr]
    void* spec = nullptr;     // [t][Lc] complex
    float* part = nullptr;
    int* counts = nullptr;    // [ncell + 1]
    int* offsets = nullptr;   // [ncell + 1]
    int* perm = nullptr;      // [n]
    double* frac = nullptr;   // [n][d] fractional grid coordinates, in perm order
    int* pcell = nullptr;     // [n] cell of each point, in perm order
    int64_t ncell = 0;
    int t = 0;
};
size_t ski_scratch_bytes(int d, const int32_t* m, int t, int64_t n);
// lo, hi: the caller's data range, or null for the range of X (and Xs).
hipError_t ski_setup(SkiOp& op, const mfgp_kernel& k, const float* X, int64_t n, const float* Xs, int64_t ms,
                     const int32_t* m, const float* lo, const float* hi, int t, void* scratch, hipStream_t s);
hipError_t ski_apply(const SkiOp& op, const float* Xc, int64_t nc, const float* Xr, int64_t nr, const float* V, int t,
                     float* out, bool with_noise, float sig2, const float* Vself, hipStream_t s);
hipError_t ski_residual(const SkiOp& op, const float* X, int64_t n, const float* B, const double* X64, int t,
                        float sig2, double* R, hipStream_t s);
// Scratch of ski_gradient (beside the SkiOp's own buffers for t columns).
size_t ski_grad_scratch_bytes(int d, const int32_t* m, int t);
// grad[j] = sum_c colw_c (W^T A_c)^T (dK_UU/dtheta_j) (W^T B_c), the kernel's
// parameters without sigma^2 in gradient order.  Synchronises.
hipError_t ski_gradient(const SkiOp& op, const mfgp_kernel& k, const float* X, int64_t n, const float* A,
                        const float* B, int t, const double* colw, double* grad, void* gscratch, hipStream_t s);

// A linear term (linear = 1) keeps the raw inputs in U (d = din, factors 1).
// Terms of a kernel sum are linked through next (see OpChain).  A product
// term (nfactors > 0) of RBF factors and at most one periodic factor is RBF
// on the concatenated features: the periodic factor's 2 din features first
// (periodic = 1), then dextra features of the RBF factors; factor[] keeps
// the caller's factor order with each factor's first feature f0.
struct GramPrep;

struct Operator {
    struct Factor {
        int periodic = 0;
        int ard = 0;
        int f0 = 0;
        int family = 0;    // mfgp_family of the factor (general products)
    };
    int family = 0;
    int d = 0;
    int din = 0;
    int dextra = 0;
    int periodic = 0;
    int linear = 0;
    int ard = 0;
    int nfactors = 0;
    Factor factor[MFGP_MAX_TERMS];
    double period = 0.0;
    const Operator* next = nullptr;
    const SkiOp* ski = nullptr;   // non-null: products by structured kernel interpolation
    int general = 0;              // a product with Matern or Linear factors (family kFamProd)
    ProdDesc pd;                  // its feature layout
    int64_t n = 0;
    float s2 = 1.0f;
    float sig2 = 0.0f;
    float fac[MFGP_MAX_D] = {};
    double ls[MFGP_MAX_D] = {};
    const float* X = nullptr;
    float* U = nullptr;
    // The Gram-form data of these points (centred features, norms, maximum
    // norm) when a solver prepared them once for all its products; null: each
    // Gram-form product prepares them itself.
    const GramPrep* gram_pre = nullptr;
};

Operator make_operator(const mfgp_kernel& k, const float* X, int64_t n, float* U);
hipError_t prescale(const Operator& op, hipStream_t s);

// The terms of a kernel (one, or a sum chained by mfgp_kernel.next) bound to
// the same points: term q reads U + n * (feature dims of the terms before it).
// Not copyable: the terms point at each other.
struct OpChain {
    Operator t[MFGP_MAX_TERMS];
    int count = 0;
    OpChain() = default;
    OpChain(const OpChain&) = delete;
    OpChain& operator=(const OpChain&) = delete;
    const Operator& head() const { return t[0]; }
};
// Feature dimension of one term (2 d periodic, d otherwise) and of the chain.
int term_feature_dim(const mfgp_kernel& k);
int chain_feature_dim(const mfgp_kernel& k);
void make_chain(OpChain& ch, const mfgp_kernel& k, const float* X, int64_t n, float* U);
hipError_t prescale_chain(const OpChain& ch, hipStream_t s);
// Gradient entries of one term without sigma^2.
int term_params(const mfgp_kernel& k);

// Products and residuals of a (possibly multi-term) operator.  scratch is
// the single-term scratch of the precision (apply_fp32_scratch_bytes or
// mfma_scratch_bytes; resid_scratch_doubles for the residual) and sum_scratch
// sum_scratch_bytes(max(m, n), t) more: the FP32 buffer of the terms after
// the first and the FP64 partials of the linear terms.  rows = NULL for the
// square product (rows are the columns' points).
size_t sum_scratch_bytes(int64_t m, int t);
hipError_t apply_sum(const Operator& cols, const Operator* rows, int64_t m, const float* V, int t,
                     float* out, bool with_noise, const float* Vself, void* scratch, void* sum_scratch,
                     int precision, hipStream_t s);
hipError_t residual_sum(const Operator& op, const float* B, const double* X64, int t, double* R,
                        double* scratch, void* sum_scratch, hipStream_t s);
// Gradient of every term's parameters, sum_c w_c A_c^T (dK/dtheta) B_c, into
// grad[0 ..) in chain order (sigma^2 excluded).
hipError_t chain_gradient(const Operator& op, const float* A, const float* B, int t, const double* colw_host,
                          double* grad, double* adj_scratch, void* sum_scratch, hipStream_t s);
// var[q] += s2_t |x_q|^2 for every linear term (the prior variance of a
// linear term at the test points U of the rows operator).
hipError_t add_linear_prior(const Operator& rows, int64_t m, float* var, hipStream_t s);
// Sum of the outputscales of the stationary terms (their prior variance).
double stationary_prior(const Operator& op);

int column_block64(int t);
hipError_t launch_pack_cols(const float* src, int lds, int c0, int tb, int64_t n, float* dst,
                            hipStream_t s);

// Scratch (in floats) that apply_f32 needs for an m-row product with t columns.
size_t apply_scratch_floats(int64_t m, int64_t n, int t);
// out[m, t] = s2 k(Ur, U) V + (with_noise ? sig2 Vself : 0), FP32 entries, FP32 sweeps.
hipError_t apply_f32(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                     float* out, bool with_noise, const float* Vself, float* scratch,
                     hipStream_t s);

// Scratch (in doubles) of residual_f64.
size_t resid_scratch_doubles(int64_t n, int t);
// R = B - K_y X64 with FP32 entries and FP64 accumulation.
hipError_t residual_f64(const Operator& op, const float* B, const double* X64, int t, double* R,
                        double* scratch, hipStream_t s);
// R -= s2 k(U, U) X64 (a later term of a sum; no noise), same arithmetic.
hipError_t residual_f64_sub(const Operator& op, const double* X64, int t, double* R, double* scratch,
                            hipStream_t s);

// FP32 sweep with the contraction on FP32 MFMA (t = 16 NT + TV, NT 1..4, TV 0..1).
bool hybrid_supported(int t);
size_t hybrid_scratch_bytes(int64_t m, int64_t n, int t);
hipError_t apply_hybrid(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                        float* out, bool with_noise, const float* Vself, void* scratch, hipStream_t s);
// FP32 RBF sweep with the squared distances on FP32 MFMA (square products,
// t = 1 or 16 k + {0, 1}; falls back in-kernel to direct differences when the
// centred norms are too large for the form's accuracy).
bool gram_supported(int t);
// Shared preparation of the Gram forms (FP32 and bf16 sweeps): the column
// mean mu of U, G [n][dg] = -2 (u - mu) zero-padded to dg = 4 (d <= 4) or 8,
// nrm [n] = |u - mu|^2 (both with rows n .. roundup(n, 64) - 1 repeating row
// n - 1) and the largest norm's float bits in *gmax; the sweeps take the Gram
// branch only while that maximum is at most kGramMaxNorm (which also keeps
// the factored entries 2^(2 g_i . g_j) <= 2^124 inside binary32, see gram.hip).
constexpr float kGramMaxNorm = 62.0f;
// Smallest n for which MFGP_FP32 and the bf16 forms take the Gram form.
constexpr int64_t kGramMinN = 32768;
struct GramPrep {
    float* G = nullptr;
    float* nrm = nullptr;
    unsigned* gmax = nullptr;
    int dg = 4;
};
size_t gram_prep_bytes(int64_t n);
hipError_t gram_prepare(const Operator& op, void* scratch, GramPrep& g, hipStream_t s);
// Rows of G and nrm for n points (n rounded up to 64).
inline int64_t gram_rows(int64_t n) { return (n + 63) / 64 * 64; }
// The same into caller-placed G (gram_rows(n) x g.dg), nrm and gmax, with
// gram_mean_bytes() of scratch for the column means.
size_t gram_mean_bytes();
hipError_t gram_prepare_into(const Operator& op, const GramPrep& g, void* mean_scratch, hipStream_t s);
size_t gram_scratch_bytes(int64_t n, int t);
hipError_t apply_gram(const Operator& op, const float* V, int t, float* out, bool with_noise, const float* Vself,
                      void* scratch, hipStream_t s);
// The fused Gram-form sweep of a two-term sum of RBF-class terms (square;
// t as gram_supported), and its scratch.
size_t gram2_scratch_bytes(int64_t n, int t);
hipError_t apply_gram2(const Operator& a, const Operator& b, const float* V, int t, float* out, bool with_noise,
                       const float* Vself, void* scratch, hipStream_t s);
// FP32-class product for precision MFGP_FP32 / _FP32_VALU / _FP32_DIRECT /
// _FP32_GRAM: the Gram form, the MFMA-contraction form or the VALU form as
// the precision, the family, the shape and the size allow (see core.hip).
size_t apply_fp32_scratch_bytes(int64_t m, int64_t n, int t, int precision);
hipError_t apply_fp32(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                      float* out, bool with_noise, const float* Vself, void* scratch, int precision,
                      hipStream_t s);
inline bool is_fp32_class(int precision) {
    return precision == MFGP_FP32 || precision == MFGP_FP32_VALU || precision == MFGP_FP32_DIRECT ||
           precision == MFGP_FP32_GRAM;
}

// BF16-MFMA tile products (precision x1 / x2).
bool precision_supported(int precision);
size_t mfma_scratch_bytes(int64_t m, int64_t n, int t, int precision);
hipError_t apply_mfma(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                      float* out, bool with_noise, const float* Vself, int precision,
                      void* scratch, hipStream_t s);

// Column norms / dots in FP64: out[c] = sum_i a[i,c] * b[i,c] (float or double inputs).
size_t dots_scratch_doubles(int64_t n, int t);
hipError_t col_dots_ff(const float* a, const float* b, int64_t n, int t, double* out_dev,
                       double* scratch, hipStream_t s);
hipError_t col_dots_dd(const double* a, const double* b, int64_t n, int t, double* out_dev,
                       double* scratch, hipStream_t s);
hipError_t col_dots_df(const double* a, const float* b, int64_t n, int t, double* out_dev,
                       double* scratch, hipStream_t s);

// Gradient adjoint pass: per-parameter sums (device, FP64) over all entries.
size_t adjoint_scratch_doubles(int64_t n, int d, int t);
hipError_t adjoint_sums(const Operator& op, const float* A, const float* B, int t,
                        const double* colw_host, double* sums_host, double* scratch,
                        hipStream_t s);

// SplitMix64 Rademacher probes.
hipError_t launch_rademacher(uint64_t seed, int64_t n, int p, float* Z, hipStream_t s);

// Optional sweep timing (timing.hip): a token from timing_begin is closed by
// timing_end with the launch's algorithmic entries and FLOP.
double sweep_flops_per_entry(int family, int d, int t, bool adjoint);
void* timing_begin(hipStream_t s);
void timing_end(void* tok, hipStream_t s, int kind, double entries, double flops);
bool timing_on();
void timing_suspend(bool on);   // while a graph is captured
void timing_phase(int which, double ms);   // 0 CG solve, 1 quadrature, 2 adjoint
enum SweepKind { kSweepF32 = 0, kSweepF64 = 1, kSweepAdjoint = 2, kSweepMfma = 3 };

// Thread-local last HIP error.
void set_last_hip_error(hipError_t e);

// Per-thread library resources (hipFFT plans of the SKI calls, rocBLAS
// handles of the preconditioned calls): released on request.
hipError_t release_fft_plans();
hipError_t release_blas_handles();
hipError_t release_cg_streams();

// General products (prod.hip): the VALU entry sweeps (FP32 and FP64
// accumulation) and the adjoint sums [G_k per feature, G_s, G_p].
hipError_t sweep_prod_f32(int D, int tb, const SweepArgs& a, hipStream_t s);
hipError_t sweep_prod_f64(int D, int tb, const SweepArgs64& a, hipStream_t s);
hipError_t adjoint_prod(const Operator& op, int tb, const float* A, int lda, int c0, const float* w_host,
                        const float* B, const SweepPlan& p, double* partial, hipStream_t s);
// var[i] += s2 k^(x_i, x_i) of a general product (its Linear factors'
// |x_i|^2; 1 without them), rows Ur [m, D].
hipError_t prod_prior_add(const Operator& op, const float* Ur, int64_t m, double s2, float* var, hipStream_t s);

}  // namespace mfgp
