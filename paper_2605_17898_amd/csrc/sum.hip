// Kernel sums and the Linear family (LightGP Sec. 3 "Kernels": the concrete
// kernels include Linear, and `+` composes `Scale`d kernels into trees).
//
// A sum k = sum_t s2_t k_t is applied term by term: the first term writes
// the product (with the noise), every later term adds into it, each with
// its own product form (the stationary and periodic terms through the
// sweeps of their precision, including the Gram form).  A linear term
// s2 x.x' is rank d: K V = s2 X (X^T V), with X^T V reduced in FP64 in a
// fixed order (128 row blocks, then the blocks in order) and the product
// formed in FP64 and rounded once.  The gradient takes every term's
// parameters in chain order: the adjoint sweep of each stationary or
// periodic term, and for a linear term
//   sum_c w_c A_c^T X X^T B_c = sum_c w_c (X^T A_c) . (X^T B_c).
#include "internal.hpp"

#include <vector>

namespace mfgp {

namespace {

constexpr int kLinBlocks = 128;

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Layout of sum_scratch: FP64 partials [kLinBlocks][MAX_D * t], two d x t
// results, then the FP32 buffer [m][t] of the terms after the first.
inline size_t lin_doubles(int t) { return static_cast<size_t>(kLinBlocks + 2) * MFGP_MAX_D * t; }

template <typename T>
__global__ void lin_xtv_partial_kernel(const float* __restrict__ U, int64_t n, int d, const T* __restrict__ V, int t,
                                       int64_t rows_per_block, double* __restrict__ part) {
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * rows_per_block;
    const int64_t j1 = j0 + rows_per_block < n ? j0 + rows_per_block : n;
    const int dt = d * t;
    for (int p = threadIdx.x; p < dt; p += blockDim.x) {
        const int k = p / t;
        const int c = p - k * t;
        double acc = 0.0;
        for (int64_t j = j0; j < j1; ++j)
            acc = fma(static_cast<double>(U[j * d + k]), static_cast<double>(V[j * t + c]), acc);
        part[static_cast<int64_t>(blockIdx.x) * dt + p] = acc;
    }
}

__global__ void lin_xtv_final_kernel(const double* __restrict__ part, int nb, int dt, double* __restrict__ xtv) {
    for (int p = threadIdx.x; p < dt; p += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[static_cast<int64_t>(b) * dt + p];
        xtv[p] = s;
    }
}

// out[i, c] = (acc ? out[i, c] : 0) + s2 sum_k Ur[i, k] xtv[k, c] + (Vself ? sig2 Vself[i, c] : 0)
__global__ void lin_apply_kernel(const float* __restrict__ Ur, int64_t m, int d, const double* __restrict__ xtv,
                                 int t, double s2, int acc, const float* __restrict__ Vself, double sig2,
                                 float* __restrict__ out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * t) return;
    const int64_t i = idx / t;
    const int c = static_cast<int>(idx - i * t);
    double v = 0.0;
    for (int k = 0; k < d; ++k) v = fma(static_cast<double>(Ur[i * d + k]), xtv[k * t + c], v);
    v *= s2;
    if (acc) v += static_cast<double>(out[idx]);
    if (Vself) v += sig2 * static_cast<double>(Vself[idx]);
    out[idx] = static_cast<float>(v);
}

// Head term: R = B - (s2 X xtx + sig2 X64); later term: R -= s2 X xtx.
__global__ void lin_resid_kernel(const float* __restrict__ U, int64_t n, int d, const double* __restrict__ xtx,
                                 int t, double s2, const float* __restrict__ B, double sig2,
                                 const double* __restrict__ X64, double* __restrict__ R) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * t) return;
    const int64_t i = idx / t;
    const int c = static_cast<int>(idx - i * t);
    double v = 0.0;
    for (int k = 0; k < d; ++k) v = fma(static_cast<double>(U[i * d + k]), xtx[k * t + c], v);
    v *= s2;
    if (B)
        R[idx] = static_cast<double>(B[idx]) - (v + sig2 * X64[idx]);
    else
        R[idx] -= v;
}

__global__ void add_f32_kernel(const float* __restrict__ a, int64_t total, float* __restrict__ out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < total) out[idx] += a[idx];
}

__global__ void linear_prior_kernel(const float* __restrict__ U, int64_t m, int d, double s2, float* __restrict__ var) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= m) return;
    double a = 0.0;
    for (int k = 0; k < d; ++k) {
        const double x = static_cast<double>(U[q * d + k]);
        a = fma(x, x, a);
    }
    var[q] = static_cast<float>(static_cast<double>(var[q]) + s2 * a);
}

inline unsigned blocks_for(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

// xtv [d][t] = X^T V for the term's points U [n][d] (FP64, fixed order).
template <typename T>
hipError_t linear_xtv(const Operator& op, const T* V, int t, double* part, double* xtv, hipStream_t s) {
    const int64_t rpb = (op.n + kLinBlocks - 1) / kLinBlocks;
    hipLaunchKernelGGL((lin_xtv_partial_kernel<T>), dim3(kLinBlocks), dim3(256), 0, s, op.U, op.n, op.d, V, t, rpb,
                       part);
    hipLaunchKernelGGL(lin_xtv_final_kernel, dim3(1), dim3(256), 0, s, part, kLinBlocks, op.d * t, xtv);
    return hipGetLastError();
}

// Lengthscale factor F_k of the adjoint sums (see adjoint.hip).
double lengthscale_factor(int family, double l) {
    const double c = family_scale(family);
    switch (family) {
        case MFGP_RBF: return 1.0 / (c * c * l);
        case MFGP_MATERN12: return 1.0 / (c * l);
        case MFGP_MATERN32: return 3.0 / (c * c * l);
        default: return (5.0 / 3.0) / (c * c * l);
    }
}

// grad[0..nl-1] lengthscales, grad[nl] s2 from the adjoint sums G_k, G_s;
// periodic family: grad[0..nl-1] lengthscales, grad[nl] the period, grad[nl+1]
// s2 from G_l, G_s, G_p (see adjoint_periodic_kernel): with c the RBF scale,
//   dk/dl_k = s2 G_l[k] / (c^2 l_k),  dk/dp = s2 (2 pi / (p^2 c^2)) G_p.
// Product term (RBF on concatenated features): G holds [G_q per feature, G_s]
// without a periodic factor and [G_l (din), G_x (dextra), G_s, G_p] with one;
// each factor's lengthscales take s2 G / (c^2 l) of its features (the two of
// each input for the periodic factor), in the caller's factor order.
int grad_from_product(const Operator& op, const double* G, double* grad) {
    const double c = family_scale(MFGP_RBF);
    const int din = op.din;
    // index of feature q's sum in G (periodic features pair into G_l)
    auto gsum = [&](int q) { return op.periodic ? G[din + (q - 2 * din)] : G[q]; };
    int off = 0;
    for (int f = 0; f < op.nfactors; ++f) {
        const Operator::Factor& fi = op.factor[f];
        const int nl = fi.ard ? din : 1;
        for (int k = 0; k < nl; ++k) grad[off + k] = 0.0;
        for (int k = 0; k < din; ++k) {
            double gk;
            if (fi.periodic)
                gk = static_cast<double>(op.s2) * G[k] / (c * c * op.ls[2 * k]);
            else
                gk = static_cast<double>(op.s2) * gsum(fi.f0 + k) / (c * c * op.ls[fi.f0 + k]);
            grad[off + (fi.ard ? k : 0)] += gk;
        }
        off += nl;
        if (fi.periodic) {
            const double two_pi = 6.283185307179586477;
            grad[off++] = static_cast<double>(op.s2) * two_pi / (op.period * op.period * c * c) *
                          G[din + op.dextra + 1];
        }
    }
    grad[off++] = op.periodic ? G[din + op.dextra] : G[op.d];
    return off;
}

// Gradient entries of a general product term from its adjoint sums
// G = [G_k per feature (D), G_s, G_p]: per factor in the caller's order its
// lengthscales (s2 F_k(l) G_k, the two circle features of each input summed
// for the periodic factor) and the period, none for Linear; then s2.
int grad_from_general_product(const Operator& op, const double* G, double* grad) {
    const double s2 = static_cast<double>(op.s2);
    const double cr = family_scale(MFGP_RBF);
    const int din = op.din;
    int off = 0;
    for (int f = 0; f < op.nfactors; ++f) {
        const Operator::Factor& fi = op.factor[f];
        if (fi.family == MFGP_LINEAR) continue;
        const int nl = fi.ard ? din : 1;
        for (int k = 0; k < nl; ++k) grad[off + k] = 0.0;
        for (int k = 0; k < din; ++k) {
            double gk;
            if (fi.periodic) {
                gk = s2 * (G[2 * k] + G[2 * k + 1]) / (cr * cr * op.ls[2 * k]);
            } else {
                gk = s2 * lengthscale_factor(fi.family, op.ls[fi.f0 + k]) * G[fi.f0 + k];
            }
            grad[off + (fi.ard ? k : 0)] += gk;
        }
        off += nl;
        if (fi.periodic) {
            const double two_pi = 6.283185307179586477;
            grad[off++] = s2 * two_pi / (op.period * op.period * cr * cr) * G[op.d + 1];
        }
    }
    grad[off++] = G[op.d];
    return off;
}

// Returns the number of entries written.
int grad_from_sums(const Operator& op, const double* G, double* grad) {
    const int ard = op.ard;
    if (op.general) return grad_from_general_product(op, G, grad);
    if (op.nfactors > 0) return grad_from_product(op, G, grad);
    if (op.periodic) {
        const int din = op.din;
        const double c = family_scale(MFGP_RBF);
        double shared = 0.0;
        for (int k = 0; k < din; ++k) {
            const double gk = static_cast<double>(op.s2) * G[k] / (c * c * op.ls[2 * k]);
            if (ard)
                grad[k] = gk;
            else
                shared += gk;
        }
        const int nl = ard ? din : 1;
        if (!ard) grad[0] = shared;
        const double two_pi = 6.283185307179586477;
        grad[nl] = static_cast<double>(op.s2) * two_pi / (op.period * op.period * c * c) * G[din + 1];
        grad[nl + 1] = G[din];
        return nl + 2;
    }
    const int d = op.d;
    double shared = 0.0;
    for (int k = 0; k < d; ++k) {
        const double gk = static_cast<double>(op.s2) * lengthscale_factor(op.family, op.ls[k]) * G[k];
        if (ard)
            grad[k] = gk;
        else
            shared += gk;
    }
    const int nl = ard ? d : 1;
    if (!ard) grad[0] = shared;
    grad[nl] = G[d];
    return nl + 1;
}

}  // namespace

size_t sum_scratch_bytes(int64_t m, int t) {
    return align256(lin_doubles(t) * sizeof(double)) + align256(static_cast<size_t>(m) * t * sizeof(float)) + 256;
}

hipError_t apply_sum(const Operator& cols, const Operator* rows, int64_t m, const float* V, int t, float* out,
                     bool with_noise, const float* Vself, void* scratch, void* sum_scratch, int precision,
                     hipStream_t s) {
    if (cols.ski) {
        const Operator* rr = rows ? rows : &cols;
        return ski_apply(*cols.ski, cols.X, cols.n, rr->X, m, V, t, out, with_noise, cols.sig2, Vself, s);
    }
    // two RBF-class terms in the Gram form: one fused sweep (one contraction)
    const Operator* nb = cols.next;
    if (!rows && nb && !nb->next && !cols.linear && !nb->linear && cols.family == MFGP_RBF &&
        nb->family == MFGP_RBF && cols.d <= 8 && nb->d <= 8 && gram_supported(t) &&
        (precision == MFGP_FP32_GRAM || (precision == MFGP_FP32 && cols.n >= kGramMinN)))
        return apply_gram2(cols, *nb, V, t, out, with_noise, Vself, scratch, s);
    double* part = static_cast<double*>(sum_scratch);
    double* xtv = part + static_cast<size_t>(kLinBlocks) * MFGP_MAX_D * t;
    float* tmp = reinterpret_cast<float*>(static_cast<char*>(sum_scratch) + align256(lin_doubles(t) * sizeof(double)));
    const Operator* r = rows ? rows : &cols;
    bool first = true;
    for (const Operator* c = &cols; c; c = c->next, r = r->next) {
        if (!r) return hipErrorInvalidValue;
        const bool noise = first && with_noise;
        hipError_t e;
        if (c->linear) {
            e = linear_xtv<float>(*c, V, t, part, xtv, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(lin_apply_kernel, dim3(blocks_for(m * t)), dim3(256), 0, s, r->U, m, c->d, xtv, t,
                               static_cast<double>(c->s2), first ? 0 : 1, noise ? Vself : nullptr,
                               static_cast<double>(c->sig2), out);
            e = hipGetLastError();
        } else {
            float* dst = first ? out : tmp;
            if (is_fp32_class(precision))
                e = apply_fp32(*c, r->U, m, V, t, dst, noise, Vself, scratch, precision, s);
            else
                e = apply_mfma(*c, r->U, m, V, t, dst, noise, Vself, precision, scratch, s);
            if (e == hipSuccess && !first) {
                hipLaunchKernelGGL(add_f32_kernel, dim3(blocks_for(m * t)), dim3(256), 0, s, tmp, m * t, out);
                e = hipGetLastError();
            }
        }
        if (e != hipSuccess) return e;
        first = false;
    }
    return hipSuccess;
}

hipError_t residual_sum(const Operator& op, const float* B, const double* X64, int t, double* R, double* scratch,
                        void* sum_scratch, hipStream_t s) {
    if (op.ski) return ski_residual(*op.ski, op.X, op.n, B, X64, t, op.sig2, R, s);
    double* part = static_cast<double*>(sum_scratch);
    double* xtv = part + static_cast<size_t>(kLinBlocks) * MFGP_MAX_D * t;
    bool first = true;
    for (const Operator* c = &op; c; c = c->next) {
        hipError_t e;
        if (c->linear) {
            e = linear_xtv<double>(*c, X64, t, part, xtv, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(lin_resid_kernel, dim3(blocks_for(c->n * t)), dim3(256), 0, s, c->U, c->n, c->d, xtv,
                               t, static_cast<double>(c->s2), first ? B : nullptr, static_cast<double>(c->sig2), X64,
                               R);
            e = hipGetLastError();
        } else if (first) {
            e = residual_f64(*c, B, X64, t, R, scratch, s);
        } else {
            e = residual_f64_sub(*c, X64, t, R, scratch, s);
        }
        if (e != hipSuccess) return e;
        first = false;
    }
    return hipSuccess;
}

hipError_t chain_gradient(const Operator& op, const float* A, const float* B, int t, const double* colw_host,
                          double* grad, double* adj_scratch, void* sum_scratch, hipStream_t s) {
    double* part = static_cast<double*>(sum_scratch);
    double* xta = part + static_cast<size_t>(kLinBlocks) * MFGP_MAX_D * t;
    double* xtb = xta + static_cast<size_t>(MFGP_MAX_D) * t;
    int off = 0;
    for (const Operator* c = &op; c; c = c->next) {
        if (c->linear) {
            hipError_t e = linear_xtv<float>(*c, A, t, part, xta, s);
            if (e == hipSuccess) e = linear_xtv<float>(*c, B, t, part, xtb, s);
            if (e != hipSuccess) return e;
            const int dt = c->d * t;
            std::vector<double> h(2 * static_cast<size_t>(dt));
            e = hipMemcpyAsync(h.data(), xta, dt * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h.data() + dt, xtb, dt * sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            double g = 0.0;
            for (int cc = 0; cc < t; ++cc) {
                double dot = 0.0;
                for (int k = 0; k < c->d; ++k) dot += h[k * t + cc] * h[dt + k * t + cc];
                g += colw_host[cc] * dot;
            }
            grad[off++] = g;
        } else {
            double sums[MFGP_MAX_D + 2];
            hipError_t e = adjoint_sums(*c, A, B, t, colw_host, sums, adj_scratch, s);
            if (e != hipSuccess) return e;
            off += grad_from_sums(*c, sums, grad + off);
        }
    }
    return hipSuccess;
}

// The point-dependent prior k(x*, x*) of Linear terms and general products.
hipError_t add_linear_prior(const Operator& rows, int64_t m, float* var, hipStream_t s) {
    for (const Operator* r = &rows; r; r = r->next) {
        hipError_t e = hipSuccess;
        if (r->general) {
            e = prod_prior_add(*r, r->U, m, static_cast<double>(r->s2), var, s);
        } else if (r->linear) {
            hipLaunchKernelGGL(linear_prior_kernel, dim3(blocks_for(m)), dim3(256), 0, s, r->U, m, r->d,
                               static_cast<double>(r->s2), var);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The constant prior s2 of the stationary terms (the others: add_linear_prior).
double stationary_prior(const Operator& op) {
    double s2 = 0.0;
    for (const Operator* c = &op; c; c = c->next)
        if (!c->linear && !c->general) s2 += static_cast<double>(c->s2);
    return s2;
}

}  // namespace mfgp
