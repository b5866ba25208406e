// Core launchers shared by every entry point: prescale, split-j planning,
// column packing, partial-sum reduction, and the FP32 / FP64-accumulated
// operator products  out = s2 k(Ur, Uc) V + sig2 V  built from the sweeps.
#include "common.hpp"
#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace mfgp {

hipError_t sweep_f32_fam0(int, int, const SweepArgs&, hipStream_t);
hipError_t sweep_f32_fam1(int, int, const SweepArgs&, hipStream_t);
hipError_t sweep_f32_fam2(int, int, const SweepArgs&, hipStream_t);
hipError_t sweep_f32_fam3(int, int, const SweepArgs&, hipStream_t);
hipError_t sweep_f64_fam0(int, int, const SweepArgs64&, hipStream_t);
hipError_t sweep_f64_fam1(int, int, const SweepArgs64&, hipStream_t);
hipError_t sweep_f64_fam2(int, int, const SweepArgs64&, hipStream_t);
hipError_t sweep_f64_fam3(int, int, const SweepArgs64&, hipStream_t);

double family_scale(int family) {
    const double log2e = 1.4426950408889634074;
    switch (family) {
        case MFGP_RBF: return std::sqrt(log2e / 2.0);
        case MFGP_MATERN12: return log2e;
        case MFGP_MATERN32: return std::sqrt(3.0) * log2e;
        case MFGP_MATERN52: return std::sqrt(5.0) * log2e;
        default: return 0.0;
    }
}

SweepPlan plan_sweep(int64_t m, int64_t n, int64_t target) {
    SweepPlan p;
    p.m = m;
    p.n = n;
    p.rowblocks = static_cast<int>((m + kBlock - 1) / kBlock);
    // Aim for ~target blocks (4096 by default: 2 dispatch rounds at 8
    // resident 256-thread blocks per CU on 256 CUs), each j-range at least
    // 256 long.
    int64_t chunks = (target + p.rowblocks - 1) / p.rowblocks;
    const int64_t max_chunks = n / 256 > 1 ? n / 256 : 1;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks > 64) chunks = 64;
    if (chunks >= 8) chunks = (chunks + 7) / 8 * 8;
    if (chunks < 1) chunks = 1;
    p.chunks = static_cast<int>(chunks);
    p.jchunk = (n + chunks - 1) / chunks;
    return p;
}

int column_block(int t) {
    static const int sizes[] = {33, 32, 17, 16, 8, 7, 6, 5, 4, 3, 2, 1};
    for (int s : sizes)
        if (s <= t) return s;
    return 1;
}

int column_block64(int t) {
    static const int sizes[] = {33, 32, 17, 16, 8, 4, 2, 1};
    for (int s : sizes)
        if (s <= t) return s;
    return 1;
}

hipError_t launch_sweep_f32(int family, int D, int tb, const SweepArgs& a, hipStream_t s) {
    if (family == kFamProd) return sweep_prod_f32(D, tb, a, s);
    switch (family) {
        case MFGP_RBF: return sweep_f32_fam0(D, tb, a, s);
        case MFGP_MATERN12: return sweep_f32_fam1(D, tb, a, s);
        case MFGP_MATERN32: return sweep_f32_fam2(D, tb, a, s);
        case MFGP_MATERN52: return sweep_f32_fam3(D, tb, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_f64acc(int family, int D, int tb, const SweepArgs64& a, hipStream_t s) {
    if (family == kFamProd) return sweep_prod_f64(D, tb, a, s);
    switch (family) {
        case MFGP_RBF: return sweep_f64_fam0(D, tb, a, s);
        case MFGP_MATERN12: return sweep_f64_fam1(D, tb, a, s);
        case MFGP_MATERN32: return sweep_f64_fam2(D, tb, a, s);
        case MFGP_MATERN52: return sweep_f64_fam3(D, tb, a, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- small kernels

struct Fac {
    float f[MFGP_MAX_D];
};

__global__ void prescale_kernel(const float* __restrict__ X, int64_t n, int d, Fac fac,
                                float* __restrict__ U) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * d) return;
    const int k = static_cast<int>(idx % d);
    U[idx] = X[idx] * fac.f[k];
}

hipError_t launch_prescale(const float* X, int64_t n, int d, const float* fac_host, float* U,
                           hipStream_t s) {
    Fac f{};
    for (int k = 0; k < d; ++k) f.f[k] = fac_host[k];
    const int64_t total = n * d;
    const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
    hipLaunchKernelGGL(prescale_kernel, dim3(blocks), dim3(256), 0, s, X, n, d, f, U);
    return hipGetLastError();
}

// dst[j, c] = src[j, c0 + c] for c < tb  (column block packing)
__global__ void pack_cols_kernel(const float* __restrict__ src, int lds, int c0, int tb,
                                 int64_t n, float* __restrict__ dst) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * tb) return;
    const int64_t j = idx / tb;
    const int c = static_cast<int>(idx % tb);
    dst[idx] = src[j * lds + c0 + c];
}

hipError_t launch_pack_cols(const float* src, int lds, int c0, int tb, int64_t n, float* dst,
                            hipStream_t s) {
    const int64_t total = n * tb;
    hipLaunchKernelGGL(pack_cols_kernel, dim3(static_cast<unsigned>((total + 255) / 256)),
                       dim3(256), 0, s, src, lds, c0, tb, n, dst);
    return hipGetLastError();
}

// out[i, c0 + c] = s2 * sum_s partial[s][i][c] + sig2 * Vself[i, c0 + c]
__global__ void reduce_f32_kernel(const float* __restrict__ partial, int chunks, int64_t m,
                                  int tb, float s2, float sig2, const float* __restrict__ Vself,
                                  int ldv, int c0, float* __restrict__ out, int ldo) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * tb) return;
    const int64_t i = idx / tb;
    const int c = static_cast<int>(idx % tb);
    double acc = 0.0;
    for (int s = 0; s < chunks; ++s) acc += static_cast<double>(partial[s * m * tb + idx]);
    double v = static_cast<double>(s2) * acc;
    if (Vself) v += static_cast<double>(sig2) * static_cast<double>(Vself[i * ldv + c0 + c]);
    out[i * ldo + c0 + c] = static_cast<float>(v);
}

// R[i, c0 + c] = B[i, c0 + c] - (s2 * sum_s partial[s][i][c] + sig2 * X[i, c0 + c])   (FP64)
__global__ void reduce_resid_kernel(const double* __restrict__ partial, int chunks, int64_t m,
                                    int tb, double s2, double sig2, const double* __restrict__ X,
                                    const float* __restrict__ B, int ld, int c0,
                                    double* __restrict__ R) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * tb) return;
    const int64_t i = idx / tb;
    const int c = static_cast<int>(idx % tb);
    double acc = 0.0;
    for (int s = 0; s < chunks; ++s) acc += partial[s * m * tb + idx];
    const int64_t o = i * ld + c0 + c;
    R[o] = static_cast<double>(B[o]) - (s2 * acc + sig2 * X[o]);
}

hipError_t reduce_partials(const float* partial, int chunks, int64_t m, int t, float s2,
                           float sig2, const float* Vself, float* out, hipStream_t s) {
    const int64_t total = m * t;
    hipLaunchKernelGGL(reduce_f32_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                       0, s, partial, chunks, m, t, s2, sig2, Vself, t, 0, out, t);
    return hipGetLastError();
}

// ---------------------------------------------------------------- operator products

// A product term of RBF factors and at most one periodic factor (the checks
// are the caller's): RBF with unit lengthscales on the concatenated features,
// the periodic block first.
// A product with Matern or Linear factors (the general product, prod.hip):
// features ordered RBF-class first (the periodic factor's circle features,
// then the RBF factors'), then each Matern factor (x c_nu / l), then each
// Linear factor (x itself); op.factor[] keeps the caller's factor order.
static Operator make_general_product(const mfgp_kernel& k, const float* X, int64_t n, float* U) {
    Operator op;
    op.family = kFamProd;
    op.general = 1;
    op.din = k.d;
    op.n = n;
    op.s2 = k.outputscale;
    op.sig2 = k.noise;
    op.X = X;
    op.U = U;
    int nf = 0;
    for (const mfgp_kernel* f = &k; f && nf < MFGP_MAX_TERMS; f = f->times, ++nf) {
        Operator::Factor& fi = op.factor[nf];
        fi.family = f->family;
        fi.periodic = f->family == MFGP_PERIODIC;
        fi.ard = f->ard ? 1 : 0;
    }
    op.nfactors = nf;
    // the four classes in layout order: periodic, RBF, Matern, Linear
    int f0 = 0;
    for (int cls = 0; cls < 4; ++cls) {
        int q = 0;
        for (const mfgp_kernel* f = &k; f && q < nf; f = f->times, ++q) {
            const int fam = f->family;
            const int fc = fam == MFGP_PERIODIC ? 0 : (fam == MFGP_RBF ? 1 : (fam == MFGP_LINEAR ? 3 : 2));
            if (fc != cls) continue;
            Operator::Factor& fi = op.factor[q];
            fi.f0 = f0;
            const int width = fi.periodic ? 2 * k.d : k.d;
            const double c = fam == MFGP_LINEAR ? 1.0 : family_scale(fi.periodic ? MFGP_RBF : fam);
            for (int e = 0; e < width; ++e) {
                const int in = fi.periodic ? e / 2 : e;
                const double l = fam == MFGP_LINEAR ? 1.0 : (f->ard ? f->lengthscale[in] : f->lengthscale[0]);
                op.fac[f0 + e] = static_cast<float>(c / l);
                op.ls[f0 + e] = l;
            }
            if (fi.periodic) {
                op.periodic = 1;
                op.period = static_cast<double>(f->period);
            }
            if (cls >= 2) {
                const int sidx = op.pd.nspec++;
                op.pd.kind[sidx] = fam;
                op.pd.f0[sidx] = f0;
                op.pd.f1[sidx] = f0 + width;
            }
            f0 += width;
        }
        if (cls == 1) op.pd.nr = f0;
    }
    op.d = f0;
    return op;
}

static Operator make_product(const mfgp_kernel& k, const float* X, int64_t n, float* U) {
    for (const mfgp_kernel* f = &k; f; f = f->times)
        if (f->family != MFGP_RBF && f->family != MFGP_PERIODIC) return make_general_product(k, X, n, U);
    Operator op;
    op.family = MFGP_RBF;
    op.din = k.d;
    op.n = n;
    op.s2 = k.outputscale;
    op.sig2 = k.noise;
    op.X = X;
    op.U = U;
    const double c = family_scale(MFGP_RBF);
    int f0 = 0;
    for (const mfgp_kernel* f = &k; f; f = f->times) {
        if (f->family != MFGP_PERIODIC) continue;
        op.periodic = 1;
        op.period = static_cast<double>(f->period);
        for (int q = 0; q < 2 * k.d; ++q) {
            const double l = f->ard ? f->lengthscale[q / 2] : f->lengthscale[0];
            op.fac[q] = static_cast<float>(c / l);
            op.ls[q] = l;
        }
        f0 = 2 * k.d;
    }
    int nf = 0;
    for (const mfgp_kernel* f = &k; f && nf < MFGP_MAX_TERMS; f = f->times, ++nf) {
        Operator::Factor& fi = op.factor[nf];
        fi.periodic = f->family == MFGP_PERIODIC;
        fi.ard = f->ard ? 1 : 0;
        if (fi.periodic) {
            fi.f0 = 0;
            continue;
        }
        fi.f0 = f0;
        for (int q = 0; q < k.d; ++q) {
            const double l = f->ard ? f->lengthscale[q] : f->lengthscale[0];
            op.fac[f0 + q] = static_cast<float>(c / l);
            op.ls[f0 + q] = l;
        }
        f0 += k.d;
    }
    op.nfactors = nf;
    op.d = f0;
    op.dextra = op.periodic ? f0 - 2 * k.d : 0;
    return op;
}

Operator make_operator(const mfgp_kernel& k, const float* X, int64_t n, float* U) {
    if (k.times) return make_product(k, X, n, U);
    Operator op;
    op.ard = k.ard ? 1 : 0;
    if (k.family == MFGP_LINEAR) {
        // the raw inputs, copied into U by prescale
        op.linear = 1;
        op.family = MFGP_LINEAR;
        op.d = op.din = k.d;
        op.n = n;
        op.s2 = k.outputscale;
        op.sig2 = k.noise;
        op.X = X;
        op.U = U;
        for (int q = 0; q < op.d; ++q) {
            op.fac[q] = 1.0f;
            op.ls[q] = 1.0;
        }
        return op;
    }
    op.periodic = k.family == MFGP_PERIODIC;
    op.family = op.periodic ? MFGP_RBF : k.family;
    op.din = k.d;
    op.d = op.periodic ? 2 * k.d : k.d;
    op.period = op.periodic ? static_cast<double>(k.period) : 0.0;
    op.n = n;
    op.s2 = k.outputscale;
    op.sig2 = k.noise;
    op.X = X;
    op.U = U;
    const double c = family_scale(op.family);
    for (int q = 0; q < op.d; ++q) {
        const int in = op.periodic ? q / 2 : q;   // both features of input k share l_k
        const double l = k.ard ? k.lengthscale[in] : k.lengthscale[0];
        op.fac[q] = static_cast<float>(c / l);
        op.ls[q] = l;
    }
    return op;
}

// U[i, 2k] = fac_2k cos(2 pi x_ik / p), U[i, 2k+1] = fac_2k+1 sin(2 pi x_ik / p):
// the periodic family's features.  The phase x / p is reduced to [-1/2, 1/2]
// and the circle functions evaluated in FP64, so the features carry only the
// final rounding to FP32.
__global__ void periodic_features_kernel(const float* __restrict__ X, int64_t n, int din,
                                         double p, Fac fac, float* __restrict__ U, int ldu) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * din) return;
    const int64_t i = idx / din;
    const int k = static_cast<int>(idx - i * din);
    double ph = static_cast<double>(X[idx]) / p;
    ph -= rint(ph);
    double sn, cs;
    sincospi(2.0 * ph, &sn, &cs);
    U[i * ldu + 2 * k] = static_cast<float>(static_cast<double>(fac.f[2 * k]) * cs);
    U[i * ldu + 2 * k + 1] = static_cast<float>(static_cast<double>(fac.f[2 * k + 1]) * sn);
}

// U[i, f0 + k] = X[i, k] fac_f0+k for k < din (an RBF factor of a product term)
__global__ void prescale_cols_kernel(const float* __restrict__ X, int64_t n, int din, Fac fac, int f0,
                                     float* __restrict__ U, int ldu) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * din) return;
    const int64_t i = idx / din;
    const int k = static_cast<int>(idx - i * din);
    U[i * ldu + f0 + k] = X[idx] * fac.f[f0 + k];
}

int term_feature_dim(const mfgp_kernel& k) {
    if (k.times) {
        int f = 0;
        for (const mfgp_kernel* q = &k; q; q = q->times) f += q->family == MFGP_PERIODIC ? 2 * k.d : k.d;
        return f;
    }
    return k.family == MFGP_PERIODIC ? 2 * k.d : k.d;
}

int chain_feature_dim(const mfgp_kernel& k) {
    int f = 0;
    for (const mfgp_kernel* t = &k; t; t = t->next) f += term_feature_dim(*t);
    return f;
}

int term_params(const mfgp_kernel& k) {
    if (k.times) {
        int p = 1;   // s2
        for (const mfgp_kernel* q = &k; q; q = q->times)
            if (q->family != MFGP_LINEAR) p += (q->ard ? k.d : 1) + (q->family == MFGP_PERIODIC ? 1 : 0);
        return p;
    }
    if (k.family == MFGP_LINEAR) return 1;
    return (k.ard ? k.d : 1) + (k.family == MFGP_PERIODIC ? 2 : 1);
}

void make_chain(OpChain& ch, const mfgp_kernel& k, const float* X, int64_t n, float* U) {
    ch.count = 0;
    int64_t off = 0;
    for (const mfgp_kernel* t = &k; t && ch.count < MFGP_MAX_TERMS; t = t->next) {
        Operator& op = ch.t[ch.count];
        op = make_operator(*t, X, n, U ? U + off * n : nullptr);
        if (ch.count > 0) {
            op.sig2 = 0.0f;   // the head's noise is the sum's
            ch.t[ch.count - 1].next = &op;
        }
        off += term_feature_dim(*t);
        ++ch.count;
    }
}

hipError_t prescale_chain(const OpChain& ch, hipStream_t s) {
    for (int q = 0; q < ch.count; ++q) {
        hipError_t e = prescale(ch.t[q], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t prescale(const Operator& op, hipStream_t s) {
    if (!op.periodic && op.nfactors == 0) return launch_prescale(op.X, op.n, op.d, op.fac, op.U, s);
    Fac f{};
    for (int q = 0; q < op.d; ++q) f.f[q] = op.fac[q];
    const int64_t total = op.n * op.din;
    const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
    if (op.periodic)
        hipLaunchKernelGGL(periodic_features_kernel, dim3(blocks), dim3(256), 0, s, op.X, op.n, op.din, op.period, f,
                           op.U, op.d);
    for (int q = 0; q < op.nfactors; ++q) {
        if (op.factor[q].periodic) continue;
        hipLaunchKernelGGL(prescale_cols_kernel, dim3(blocks), dim3(256), 0, s, op.X, op.n, op.din, f,
                           op.factor[q].f0, op.U, op.d);
    }
    return hipGetLastError();
}

size_t apply_scratch_floats(int64_t m, int64_t n, int t) {
    const SweepPlan p = plan_sweep(m, n);
    const int tb = column_block(t);
    const size_t part = static_cast<size_t>(p.chunks) * m * tb;
    const size_t pack = (tb == t) ? 0 : static_cast<size_t>(n) * tb;
    return part + pack + 64;
}

hipError_t apply_f32(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                     float* out, bool with_noise, const float* Vself, float* scratch,
                     hipStream_t s) {
    const SweepPlan plan = plan_sweep(m, op.n);
    const int tb0 = column_block(t);
    float* partial = scratch;
    float* pack = scratch + ((static_cast<size_t>(plan.chunks) * m * tb0 + 63) / 64) * 64;
    for (int c0 = 0; c0 < t;) {
        const int tb = column_block(t - c0);
        const float* vb = V;
        if (tb != t) {
            hipError_t e = launch_pack_cols(V, t, c0, tb, op.n, pack, s);
            if (e != hipSuccess) return e;
            vb = pack;
        }
        SweepArgs a{Ur, op.U, vb, m, op.n, partial, plan, op.general ? &op.pd : nullptr};
        void* tok = timing_begin(s);
        hipError_t e = launch_sweep_f32(op.family, op.d, tb, a, s);
        const double ent = static_cast<double>(m) * static_cast<double>(op.n);
        timing_end(tok, s, kSweepF32, ent, ent * sweep_flops_per_entry(op.family, op.d, tb, false));
        if (e != hipSuccess) return e;
        const int64_t total = m * tb;
        hipLaunchKernelGGL(reduce_f32_kernel, dim3(static_cast<unsigned>((total + 255) / 256)),
                           dim3(256), 0, s, partial, plan.chunks, m, tb, op.s2,
                           with_noise ? op.sig2 : 0.0f, with_noise ? Vself : nullptr, t, c0, out,
                           t);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        c0 += tb;
    }
    return hipSuccess;
}

// Form selection of the FP32-class products.  MFGP_FP32 takes the Gram form
// for square RBF products of at least kGramMinN rows (below that its four
// preparation launches cost about what it saves: 0.130 against 0.126 ms at
// n = 20000, t = 1; 0.51 against 0.60 ms at n = 50000), else the MFMA-
// contraction form where t = 16 k + {0, 1}, else the VALU form;
// MFGP_FP32_GRAM takes the Gram form at any size, MFGP_FP32_DIRECT never.

static bool use_gram(const Operator& op, const float* Ur, int64_t m, int t, int precision) {
    if (precision != MFGP_FP32 && precision != MFGP_FP32_GRAM) return false;
    if (op.family != MFGP_RBF || Ur != op.U || m != op.n || !gram_supported(t)) return false;
    return precision == MFGP_FP32_GRAM || op.n >= kGramMinN;
}

size_t apply_fp32_scratch_bytes(int64_t m, int64_t n, int t, int precision) {
    size_t b = apply_scratch_floats(m, n, t) * sizeof(float);
    if (precision != MFGP_FP32_VALU && hybrid_supported(t)) b = std::max(b, hybrid_scratch_bytes(m, n, t));
    if ((precision == MFGP_FP32 || precision == MFGP_FP32_GRAM) && m == n && gram_supported(t))
        b = std::max(b, std::max(gram_scratch_bytes(n, t), gram2_scratch_bytes(n, t)));
    return b;
}

hipError_t apply_fp32(const Operator& op, const float* Ur, int64_t m, const float* V, int t,
                      float* out, bool with_noise, const float* Vself, void* scratch, int precision,
                      hipStream_t s) {
    if (op.general) return apply_f32(op, Ur, m, V, t, out, with_noise, Vself, static_cast<float*>(scratch), s);
    if (use_gram(op, Ur, m, t, precision)) return apply_gram(op, V, t, out, with_noise, Vself, scratch, s);
    if (precision != MFGP_FP32_VALU && hybrid_supported(t))
        return apply_hybrid(op, Ur, m, V, t, out, with_noise, Vself, scratch, s);
    return apply_f32(op, Ur, m, V, t, out, with_noise, Vself, static_cast<float*>(scratch), s);
}

size_t resid_scratch_doubles(int64_t n, int t) {
    const SweepPlan p = plan_sweep(n, n);
    const int tb = column_block64(t);
    return static_cast<size_t>(p.chunks) * n * tb + 64;
}

// R[i, c0 + c] -= s2 * sum_s partial[s][i][c]   (FP64; a later term of a sum)
__global__ void reduce_resid_sub_kernel(const double* __restrict__ partial, int chunks, int64_t m, int tb,
                                        double s2, int ld, int c0, double* __restrict__ R) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * tb) return;
    const int64_t i = idx / tb;
    const int c = static_cast<int>(idx % tb);
    double acc = 0.0;
    for (int s = 0; s < chunks; ++s) acc += partial[s * m * tb + idx];
    R[i * ld + c0 + c] -= s2 * acc;
}

hipError_t residual_f64_sub(const Operator& op, const double* X64, int t, double* R, double* scratch,
                            hipStream_t s) {
    const SweepPlan plan = plan_sweep(op.n, op.n);
    for (int c0 = 0; c0 < t;) {
        const int tb = column_block64(t - c0);
        SweepArgs64 a{op.U, op.U, X64 + c0, t, op.n, op.n, scratch, plan, op.general ? &op.pd : nullptr};
        void* tok = timing_begin(s);
        hipError_t e = launch_sweep_f64acc(op.family, op.d, tb, a, s);
        const double ent = static_cast<double>(op.n) * static_cast<double>(op.n);
        timing_end(tok, s, kSweepF64, ent, ent * sweep_flops_per_entry(op.family, op.d, tb, false));
        if (e != hipSuccess) return e;
        const int64_t total = op.n * tb;
        hipLaunchKernelGGL(reduce_resid_sub_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                           0, s, scratch, plan.chunks, op.n, tb, static_cast<double>(op.s2), t, c0, R);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        c0 += tb;
    }
    return hipSuccess;
}

hipError_t residual_f64(const Operator& op, const float* B, const double* X64, int t, double* R,
                        double* scratch, hipStream_t s) {
    const SweepPlan plan = plan_sweep(op.n, op.n);
    for (int c0 = 0; c0 < t;) {
        const int tb = column_block64(t - c0);
        SweepArgs64 a{op.U, op.U, X64 + c0, t, op.n, op.n, scratch, plan, op.general ? &op.pd : nullptr};
        void* tok = timing_begin(s);
        hipError_t e = launch_sweep_f64acc(op.family, op.d, tb, a, s);
        const double ent = static_cast<double>(op.n) * static_cast<double>(op.n);
        timing_end(tok, s, kSweepF64, ent, ent * sweep_flops_per_entry(op.family, op.d, tb, false));
        if (e != hipSuccess) return e;
        const int64_t total = op.n * tb;
        hipLaunchKernelGGL(reduce_resid_kernel, dim3(static_cast<unsigned>((total + 255) / 256)),
                           dim3(256), 0, s, scratch, plan.chunks, op.n, tb,
                           static_cast<double>(op.s2), static_cast<double>(op.sig2), X64, B, t,
                           c0, R);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        c0 += tb;
    }
    return hipSuccess;
}

}  // namespace mfgp
