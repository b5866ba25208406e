// Conjugate-gradient driver on the matrix-free operator (LightGP Sec. 2
// "CG-based inference": CG needs only K_y v; Sec. 5: the CG loop is plain,
// unpreconditioned; several columns are stepped together here).
//
// Per iteration (all on the caller's stream):
//   AP = K_y P                      entry sweeps + reduce   (the O(n^2 t) step)
//   pap = diag(P^T AP)              FP64 striped dots
//   alpha = rr / pap                FP64, one block
//   X += alpha P (FP64), R -= alpha AP, rr_new = diag(R^T R)
//   beta = rr_new / rr, log (alpha, beta), freeze converged columns
//   P = R + beta P
// Every `check_every` iterations the host reads the active flags.  When no
// column is active the true residual B - K_y X is recomputed with FP64
// accumulation (X is FP64), and columns above tolerance restart from it
// (iterative refinement).  While iterating, a column whose recurrence
// residual has fallen tenfold since its last true residual has r replaced by
// the recomputed true residual (residual replacement, van der Vorst & Ye
// 2000), and its direction re-formed from it: p = r_new + beta p_prev.  This
// bounds the drift between the recurrence and the true residual that an
// inexact product (FP32, and more so the BF16 forms) causes, without
// discarding the Krylov space as a restart does.  It is only sound while the
// drift is small: a column whose recurrence has moved more than 10% away from
// its true residual (very ill-conditioned operators, where FP32 drift grows
// by about eps * cond per step) is left to finish its cycle and is refined.  The FP64 solution is what
// lets the recomputed residual reach 1e-6: an FP32-rounded solution alone
// floors at a few 1e-6.
#include "cg.hpp"
#include "precond.hpp"
#include "stall.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

namespace mfgp {

// Residual replacement keeps the direction only while the recurrence residual
// is within 10% of the true one: |r_true - r_rec|^2 <= 1e-2 |r_true|^2.
constexpr double kMaxDrift2 = 1e-2;
constexpr int kMaxReplaceGap = 2;   // largest check interval with replacement

// Flags of a cold start (x = 0, r = p = b); keep_iters keeps the iteration
// counts of an earlier start on another product form.
__global__ void cg_init_flags_kernel(CgState st, int t, double tol2, int keep_iters) {
    for (int c = threadIdx.x; c < t; c += blockDim.x) {
        const bool finite = isfinite(st.bnorm2[c]) && isfinite(st.rr[c]);
        const bool go = finite && st.bnorm2[c] > 0.0 && st.rr[c] > tol2 * st.bnorm2[c];
        st.active[c] = go ? 1 : 0;
        st.status[c] = finite ? MFGP_OK : MFGP_BREAKDOWN;
        if (!keep_iters) st.iters[c] = 0;
        st.lanlen[c] = 0;
        st.alpha[c] = 0.0;
        st.beta[c] = 0.0;
    }
}

CgBufs carve_cg(Carver& cv, int64_t n, int t, int precision) {
    CgBufs b;
    const size_t nt = static_cast<size_t>(n) * t;
    b.R = cv.take<float>(nt);
    b.P = cv.take<float>(nt);
    b.AP = cv.take<float>(nt);
    b.R64 = cv.take<double>(nt);
    b.scal = cv.take<double>(8 * static_cast<size_t>(t));
    b.ints = cv.take<int>(6 * static_cast<size_t>(t));
    b.dots = cv.take<double>(dots_scratch_doubles(n, t));
    b.resid = cv.take<double>(resid_scratch_doubles(n, t));
    // room for the product forms the solver may fall back to (stall.hpp)
    size_t apply = 0;
    for (int p = precision; p >= 0; p = more_accurate_precision(p))
        apply = std::max(apply, is_fp32_class(p) ? apply_fp32_scratch_bytes(n, n, t, p)
                                                 : mfma_scratch_bytes(n, n, t, p));
    b.apply = reinterpret_cast<float*>(cv.take<char>(apply));
    b.sum = cv.take<char>(sum_scratch_bytes(n, t));
    b.gram = n >= kGramMinN ? static_cast<void*>(cv.take<char>(gram_prep_bytes(n))) : nullptr;
    return b;
}

// The operator of a solve's products: op itself, with the Gram-form data of
// its points prepared once into b.gram when the products may take the Gram
// form (an RBF-class single term at n >= kGramMinN; the points do not change
// during the solve).
static hipError_t solve_operator(const Operator& op, const CgBufs& b, Operator& opg, GramPrep& pre,
                                 hipStream_t s) {
    opg = op;
    if (!b.gram || op.ski || op.general || op.family != MFGP_RBF || op.d < 1 || op.d > 8 || op.n < kGramMinN)
        return hipSuccess;
    hipError_t e = gram_prepare(op, b.gram, pre, s);
    if (e == hipSuccess) opg.gram_pre = &pre;
    return e;
}

CgBufs carve_cg_vectors(Carver& cv, int64_t n, int t) {
    CgBufs b;
    const size_t nt = static_cast<size_t>(n) * t;
    b.R = cv.take<float>(nt);
    b.P = cv.take<float>(nt);
    b.AP = cv.take<float>(nt);
    b.R64 = cv.take<double>(nt);
    b.scal = cv.take<double>(8 * static_cast<size_t>(t));
    b.ints = cv.take<int>(6 * static_cast<size_t>(t));
    b.dots = cv.take<double>(dots_scratch_doubles(n, t));
    return b;
}

static CgState make_state(const CgBufs& b, double* X, int t, double* coeff) {
    CgState st;
    st.x = X;
    st.r = b.R;
    st.p = b.P;
    st.ap = b.AP;
    st.rr = b.scal;
    st.bnorm2 = b.scal + t;
    st.pap = b.scal + 2 * t;
    st.alpha = b.scal + 3 * t;
    st.beta = b.scal + 4 * t;
    st.rrn = b.scal + 7 * t;
    st.active = b.ints;
    st.status = b.ints + t;
    st.iters = b.ints + 2 * t;
    st.lanlen = b.ints + 3 * t;
    st.coeff = coeff;
    return st;
}

static hipError_t apply_op(const Operator& op, const float* V, int t, float* out, int precision,
                           const CgBufs& b, hipStream_t s) {
    return apply_sum(op, nullptr, op.n, V, t, out, true, V, b.apply, b.sum, precision, s);
}

// Capture streams for the graph-replayed iterations: one per device and host
// thread (non-blocking, default priority), created on first use and kept
// until the thread releases them (release_cg_streams) or ends.  The caller's
// stream may be the legacy NULL stream, which cannot be captured; the graph
// recorded on this stream is launched on the caller's.
static thread_local std::map<int, hipStream_t> cap_streams;

static hipStream_t capture_stream() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto it = cap_streams.find(dev);
    if (it == cap_streams.end()) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
        it = cap_streams.emplace(dev, cs).first;
    }
    return it->second;
}

// The captured iterations of one solve: re-captured when the product form or
// the Lanczos recording changes (both are kernel arguments), destroyed with
// the solve.
struct IterGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int precision = -1, log = -1;
    void drop() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~IterGraph() { drop(); }
};

#define CG_CHECK(expr)                         \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) {                \
            set_last_hip_error(e_);            \
            return MFGP_ERR_HIP;               \
        }                                      \
    } while (0)

int cg_run(const Operator& op, const float* B, int t, double* X, const mfgp_cg_opts& o,
           mfgp_cg_info* info, double* coeff, int max_iter, const CgBufs& b, hipStream_t s) {
    const int64_t n = op.n;
    const int64_t nt = n * t;
    const double tol = o.tol;
    const int max_refine = o.max_refine >= 0 ? o.max_refine : 8;
    int check_every = o.check_every;
    if (check_every <= 0) {
        // entry-columns of one product: N^2 t for the sweeps; for structured
        // kernel interpolation its O(N 4^D + L log L) per column
        double work = static_cast<double>(n) * static_cast<double>(n) * t;
        if (op.ski) {
            const double L = static_cast<double>(op.ski->g.Lr);
            work = (static_cast<double>(n) * (1 << (2 * op.ski->g.d)) + L * std::log2(L)) * t;
        }
        check_every = work >= 1e9 ? 2 : (work >= 1e8 ? 4 : 8);
    }
    // Residual replacement only when the host sees every iteration or every
    // other one: with longer gaps it destabilised FP32 CG on ill-conditioned
    // 1-d problems (cond ~ 1e6) even at 1% drift, while plain cycles with
    // refinement converged in as many iterations.
    const bool may_replace = !o.no_replacement && check_every <= kMaxReplaceGap;
    // Launch-bound solves (checks 4 or more iterations apart): the iterations
    // between checks are captured once and replayed (not with SKI operators,
    // whose products call hipFFT).
    const bool use_graph = !o.no_graph && check_every >= 4 && !op.ski;
    IterGraph ig;
    CgState st = make_state(b, X, t, coeff);
    Operator opg;
    GramPrep gpre;
    CG_CHECK(solve_operator(op, b, opg, gpre, s));
    double* tmp = b.scal + 5 * t;     // [t] scratch scalars
    double* relt = b.scal + 6 * t;    // [t] true relative residual
    int* restart = b.ints + 4 * t;    // [t]

    CG_CHECK(col_dots_ff(B, B, n, t, st.bnorm2, b.dots, s));
    if (o.warm_start) {
        CG_CHECK(residual_sum(op, B, X, t, b.R64, b.resid, b.sum, s));
        CG_CHECK(f64_to_f32(b.R64, st.r, nt, s));
        CG_CHECK(copy2_f32(st.r, st.r, st.p, nt, s));
    } else {
        CG_CHECK(fill_f64(X, nt, 0.0, s));
        CG_CHECK(copy2_f32(B, st.r, st.p, nt, s));
    }
    CG_CHECK(col_dots_ff(st.r, st.r, n, t, st.rr, b.dots, s));
    hipLaunchKernelGGL(cg_init_flags_kernel, dim3(1), dim3(256), 0, s, st, t, tol * tol, 0);
    CG_CHECK(hipGetLastError());

    std::vector<int> h_active(t), h_iters(t), h_status(t), h_restart(t), h_refine(t, 0), h_lan(t);
    std::vector<double> h_relt(t), h_rr(t), h_b2(t), h_rep(t, 0.0);
    std::vector<int> h_flag(t, 0), h_norepl(t, 0), h_nrep(t, 0), h_skips(t, 0);
    std::vector<double> h_cross(t);
    // stagnation and precision fallback (stall.hpp): per-column trackers, the
    // true residual at each cycle's start, cycles ended by stagnation
    std::vector<StallTracker> h_stall(t);
    std::vector<double> h_t0(t, 1.0);
    std::vector<int> h_nstall(t, 0), h_gaveup(t, 0), h_stalled(t, 0);
    int precision = o.precision;
    const bool log_wanted = !o.warm_start && coeff;
    int log_coeffs = log_wanted ? 1 : 0;
    CG_CHECK(hipMemcpyAsync(h_rep.data(), st.rr, t * sizeof(double), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipMemcpyAsync(h_b2.data(), st.bnorm2, t * sizeof(double), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipStreamSynchronize(s));
    for (int c = 0; c < t; ++c) {
        h_stall[c].begin(0, h_rep[c]);
        if (h_b2[c] > 0.0) h_t0[c] = std::sqrt(h_rep[c] / h_b2[c]);
    }
    const int report_every = o.progress_every > 0 ? o.progress_every : 100;
    int next_report = report_every;
    int steps = 0;   // iterations run by the solver (every cycle; all columns advance together)

    for (;;) {
        CG_CHECK(hipMemcpyAsync(h_active.data(), st.active, t * sizeof(int), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipMemcpyAsync(h_iters.data(), st.iters, t * sizeof(int), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipMemcpyAsync(h_rr.data(), st.rr, t * sizeof(double), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipStreamSynchronize(s));
        // A column whose recurrence has stagnated ends its cycle here; when
        // that moves the solve to a more accurate form, every column's cycle
        // ends with it (they share the product, and the rest would only run
        // on into the same floor while the stopped column waits).
        const bool has_next = !op.ski && more_accurate_precision(precision) >= 0;
        bool stop = false;
        for (int c = 0; c < t; ++c) {
            if (!h_active[c] || h_iters[c] >= max_iter) continue;
            if (h_stall[c].update(h_iters[c], h_rr[c])) {
                h_active[c] = 0;
                h_nstall[c] += 1;
                h_stalled[c] = 1;
                stop = true;
            }
        }
        if (stop && has_next) std::fill(h_active.begin(), h_active.end(), 0);
        if (stop)
            CG_CHECK(hipMemcpyAsync(st.active, h_active.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
        // A column whose residual norm fell tenfold since its last true residual
        // triggers a replacement; every active column that fell at least 1.5x
        // joins it, so the columns of a block share the recomputations.
        bool any = false, replace = false;
        for (int c = 0; c < t; ++c) {
            const bool act = h_active[c] && h_iters[c] < max_iter;
            any = any || act;
            const bool can = act && !h_norepl[c] && may_replace;
            replace = replace || (can && h_rr[c] <= 0.01 * h_rep[c]);
            h_flag[c] = (can && h_rr[c] <= 0.44 * h_rep[c]) ? 1 : 0;
        }
        if (replace) {
            CG_CHECK(residual_sum(op, B, X, t, b.R64, b.resid, b.sum, s));
            // drift d = r_true - r_rec: |d|^2 = |r_true|^2 + |r_rec|^2 - 2 r_true^T r_rec
            CG_CHECK(col_dots_dd(b.R64, b.R64, n, t, tmp, b.dots, s));
            CG_CHECK(col_dots_df(b.R64, st.r, n, t, tmp + t, b.dots, s));
            CG_CHECK(hipMemcpyAsync(h_relt.data(), tmp, t * sizeof(double), hipMemcpyDeviceToHost, s));
            CG_CHECK(hipMemcpyAsync(h_cross.data(), tmp + t, t * sizeof(double), hipMemcpyDeviceToHost, s));
            CG_CHECK(hipStreamSynchronize(s));
            bool ended = false;
            for (int c = 0; c < t; ++c) {
                if (!h_flag[c]) continue;
                const double drift2 = h_relt[c] + h_rr[c] - 2.0 * h_cross[c];
                if (!(drift2 <= kMaxDrift2 * h_relt[c])) {
                    // the recurrence has left the true residual
                    h_flag[c] = 0;
                    const double tr = h_b2[c] > 0.0 ? std::sqrt(h_relt[c] / h_b2[c]) : 0.0;
                    if (has_next && cycle_wants_fallback(false, h_t0[c], tr, tol)) {
                        // at this form's floor, far above tol: end the cycle, take the next form
                        h_active[c] = 0;
                        h_nstall[c] += 1;
                        h_stalled[c] = 1;
                        ended = true;
                    } else {
                        h_norepl[c] = 1;    // run this cycle out and refine instead
                        h_skips[c] += 1;
                    }
                } else {
                    h_nrep[c] += 1;
                }
            }
            if (ended) {   // the form changes: every column's cycle ends here
                std::fill(h_active.begin(), h_active.end(), 0);
                CG_CHECK(hipMemcpyAsync(st.active, h_active.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
                any = false;
            }
            CG_CHECK(hipMemcpyAsync(restart, h_flag.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
            CG_CHECK(cg_replace(st, b.R64, n, t, restart, b.dots, tmp, s));
            CG_CHECK(hipMemcpyAsync(h_rr.data(), st.rr, t * sizeof(double), hipMemcpyDeviceToHost, s));
            CG_CHECK(hipStreamSynchronize(s));
            for (int c = 0; c < t; ++c)
                if (h_flag[c]) h_rep[c] = h_rr[c];
        }
        if (o.progress && steps >= next_report) {
            o.progress(o.progress_user, steps, worst_recurrence(h_active, h_rr, h_b2));
            while (next_report <= steps) next_report += report_every;
        }
        if (any) {
            steps += check_every;
            auto iterate = [&](hipStream_t q) -> hipError_t {
                for (int k = 0; k < check_every; ++k) {
                    hipError_t e = apply_op(opg, st.p, t, st.ap, precision, b, q);
                    if (e == hipSuccess) e = cg_pap_alpha(st, n, t, b.dots, q);
                    if (e == hipSuccess) e = cg_update_and_beta(st, n, t, b.dots, tol, log_coeffs, max_iter, q);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            };
            if (use_graph) {
                if (!ig.exec || ig.precision != precision || ig.log != log_coeffs) {
                    ig.drop();
                    hipStream_t cs = capture_stream();
                    if (!cs) CG_CHECK(hipErrorOutOfMemory);
                    CG_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                    timing_suspend(true);   // no event records inside the graph
                    const hipError_t ce = iterate(cs);
                    timing_suspend(false);
                    const hipError_t ee = hipStreamEndCapture(cs, &ig.graph);
                    CG_CHECK(ce);
                    CG_CHECK(ee);
                    CG_CHECK(hipGraphInstantiate(&ig.exec, ig.graph, nullptr, nullptr, 0));
                    ig.precision = precision;
                    ig.log = log_coeffs;
                }
                CG_CHECK(hipGraphLaunch(ig.exec, s));
            } else {
                CG_CHECK(iterate(s));
            }
            continue;
        }
        // Every column stopped: recompute the true residual in FP64.
        CG_CHECK(residual_sum(op, B, X, t, b.R64, b.resid, b.sum, s));
        CG_CHECK(col_dots_dd(b.R64, b.R64, n, t, tmp, b.dots, s));
        CG_CHECK(hipMemcpyAsync(h_relt.data(), tmp, t * sizeof(double), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipMemcpyAsync(h_b2.data(), st.bnorm2, t * sizeof(double), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipMemcpyAsync(h_status.data(), st.status, t * sizeof(int), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipStreamSynchronize(s));
        bool again = false, fallback = false;
        const int next_form = op.ski ? -1 : more_accurate_precision(precision);
        bool revive = false;
        for (int c = 0; c < t; ++c) {
            h_relt[c] = h_b2[c] > 0.0 ? std::sqrt(h_relt[c] / h_b2[c]) : 0.0;
            // p^T K_y p <= 0 cannot happen for the SPD K_y: a breakdown with a
            // finite iterate comes from an inexact product form, and the
            // next more accurate form continues from that iterate
            if (h_status[c] == MFGP_BREAKDOWN && next_form >= 0 && std::isfinite(h_relt[c]) &&
                !(h_relt[c] <= tol) && h_refine[c] < max_refine && h_iters[c] < max_iter) {
                h_status[c] = MFGP_OK;
                fallback = revive = true;
            }
            bool need = h_status[c] == MFGP_OK && !(h_relt[c] <= tol) && std::isfinite(h_relt[c]) &&
                        h_refine[c] < max_refine && h_iters[c] < max_iter && !h_gaveup[c];
            if (need && next_form >= 0 && cycle_wants_fallback(h_stalled[c], h_t0[c], h_relt[c], tol)) fallback = true;
            if (need && next_form < 0 && cycle_gave_nothing(h_t0[c], h_relt[c])) {
                h_gaveup[c] = 1;     // the last form cannot improve this column
                need = false;
            }
            h_restart[c] = need ? 1 : 0;
            if (need) {
                h_refine[c] += 1;
                again = true;
            }
        }
        if (!again) break;
        if (fallback) precision = next_form;
        if (fallback && log_wanted) {
            // The recorded tridiagonal (the SLQ log-determinant) belongs to
            // the form just left: solve again from x = 0 on the new form and
            // record it anew, so that it describes the operator the solution
            // converges on.  Every column restarts (the iterate is dropped).
            CG_CHECK(fill_f64(X, nt, 0.0, s));
            CG_CHECK(copy2_f32(B, st.r, st.p, nt, s));
            CG_CHECK(col_dots_ff(st.r, st.r, n, t, st.rr, b.dots, s));
            hipLaunchKernelGGL(cg_init_flags_kernel, dim3(1), dim3(256), 0, s, st, t, tol * tol, 1);
            CG_CHECK(hipGetLastError());
            CG_CHECK(hipMemcpyAsync(h_rep.data(), st.rr, t * sizeof(double), hipMemcpyDeviceToHost, s));
            CG_CHECK(hipStreamSynchronize(s));
            for (int c = 0; c < t; ++c) {
                h_refine[c] += h_restart[c] ? 0 : 1;   // every column restarts
                h_norepl[c] = 0;
                h_stall[c].begin(h_iters[c], h_rep[c]);
                h_t0[c] = h_b2[c] > 0.0 ? std::sqrt(h_rep[c] / h_b2[c]) : 1.0;
                h_stalled[c] = 0;
                h_gaveup[c] = 0;
            }
            log_coeffs = 1;
            continue;
        }
        if (revive)
            CG_CHECK(hipMemcpyAsync(st.status, h_status.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
        CG_CHECK(hipMemcpyAsync(restart, h_restart.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
        CG_CHECK(cg_restart(st, b.R64, n, t, restart, s));
        CG_CHECK(col_dots_ff(st.r, st.r, n, t, tmp, b.dots, s));
        CG_CHECK(cg_activate(st, t, restart, tmp, s));
        CG_CHECK(hipMemcpyAsync(h_rep.data(), tmp, t * sizeof(double), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipStreamSynchronize(s));
        for (int c = 0; c < t; ++c) {
            if (!h_restart[c]) continue;
            h_norepl[c] = 0;   // a fresh cycle starts without drift
            h_stall[c].begin(h_iters[c], h_rep[c]);
            h_t0[c] = h_relt[c];
            h_stalled[c] = 0;
        }
        log_coeffs = 0;  // the Lanczos tridiagonal belongs to the first cycle only
    }

    CG_CHECK(hipMemcpyAsync(h_rr.data(), st.rr, t * sizeof(double), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipMemcpyAsync(h_lan.data(), st.lanlen, t * sizeof(int), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipMemcpyAsync(h_iters.data(), st.iters, t * sizeof(int), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipMemcpyAsync(relt, h_relt.data(), t * sizeof(double), hipMemcpyHostToDevice, s));
    CG_CHECK(hipStreamSynchronize(s));
    int worst = MFGP_OK;
    for (int c = 0; c < t; ++c) {
        int stc = h_status[c];
        if (stc == MFGP_OK && !(h_relt[c] <= tol)) stc = MFGP_NOT_CONVERGED;
        if (stc == MFGP_BREAKDOWN)
            worst = MFGP_BREAKDOWN;
        else if (stc == MFGP_NOT_CONVERGED && worst == MFGP_OK)
            worst = MFGP_NOT_CONVERGED;
        if (info) {
            info[c].iters = h_iters[c];
            info[c].lanczos_len = h_lan[c];
            info[c].refinements = h_refine[c];
            info[c].status = stc;
            info[c].rel_resid_recurrence = h_b2[c] > 0.0 ? std::sqrt(h_rr[c] / h_b2[c]) : 0.0;
            info[c].rel_resid_true = h_relt[c];
            info[c].replacements = h_nrep[c];
            info[c].drift_skips = h_skips[c];
            info[c].stalls = h_nstall[c];
            info[c].precision = precision;
        }
    }
    return worst;
}


// ---------------------------------------------------------------- preconditioned CG

static inline unsigned nblk(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

// rz = r^T z (the PCG inner product) drives alpha and beta; rr = r^T r the
// stopping rule.  st.rr holds rz so that cg_pap_alpha computes rz / p^T A p.
__global__ void pcg_beta_kernel(CgState st, int t, const double* __restrict__ rzn_all,
                                const double* __restrict__ rrn_all, double tol2, int log_coeffs, int max_iter) {
    for (int c = threadIdx.x; c < t; c += blockDim.x) {
        double b = 0.0;
        if (st.active[c]) {
            const double rzn = rzn_all[c], rrn = rrn_all[c];
            b = rzn / st.rr[c];
            if (log_coeffs && st.coeff && st.lanlen[c] < max_iter) {
                double* cf = st.coeff + (static_cast<int64_t>(c) * max_iter + st.lanlen[c]) * 2;
                cf[0] = st.alpha[c];
                cf[1] = b;
                st.lanlen[c] += 1;
            }
            st.iters[c] += 1;
            st.rr[c] = rzn;
            st.rrn[c] = rrn;
            if (!isfinite(rzn) || !isfinite(rrn)) {
                st.status[c] = MFGP_BREAKDOWN;
                st.active[c] = 0;
            } else if (rrn <= tol2 * st.bnorm2[c] || st.iters[c] >= max_iter) {
                st.active[c] = 0;
            }
        }
        st.beta[c] = b;
    }
}

// p = z + beta p for active columns (all columns when `all`, with beta 0: p = z).
__global__ void pcg_p_kernel(CgState st, const float* __restrict__ Z, int64_t total, int t,
                             const int* __restrict__ only) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = static_cast<int>(idx % t);
    if (only) {
        if (only[c]) st.p[idx] = Z[idx];
        return;
    }
    if (!st.active[c]) return;
    st.p[idx] = fmaf(static_cast<float>(st.beta[c]), st.p[idx], Z[idx]);
}

__global__ void pcg_init_kernel(CgState st, int t, double tol2, const double* __restrict__ rr0,
                                double* __restrict__ rz0, int keep_iters) {
    for (int c = threadIdx.x; c < t; c += blockDim.x) {
        const bool finite = isfinite(st.bnorm2[c]) && isfinite(st.rr[c]) && isfinite(rr0[c]);
        const bool go = finite && st.bnorm2[c] > 0.0 && rr0[c] > tol2 * st.bnorm2[c];
        st.active[c] = go ? 1 : 0;
        st.status[c] = finite ? MFGP_OK : MFGP_BREAKDOWN;
        if (!keep_iters) st.iters[c] = 0;
        st.lanlen[c] = 0;
        st.alpha[c] = 0.0;
        st.beta[c] = 0.0;
        st.rrn[c] = rr0[c];
        rz0[c] = st.rr[c];
    }
}

// Refinement restart of flagged columns: rz = rz_new, rr = rr_new, active again.
__global__ void pcg_activate_kernel(CgState st, int t, const int* __restrict__ restart,
                                    const double* __restrict__ rz_new, const double* __restrict__ rr_new) {
    for (int c = threadIdx.x; c < t; c += blockDim.x) {
        if (restart[c]) {
            st.active[c] = rr_new[c] > 0.0 ? 1 : 0;
            st.rr[c] = rz_new[c];
            st.rrn[c] = rr_new[c];
        }
    }
}

PcgBufs carve_pcg(Carver& cv, int64_t n, int k, int t) {
    PcgBufs pb;
    pb.Zv = cv.take<float>(static_cast<size_t>(n) * t);
    pb.pc = cv.take<double>(pc_scratch_doubles(n, k, t));
    pb.rz0 = cv.take<double>(static_cast<size_t>(t));
    return pb;
}

int pcg_run(const Operator& op, const Precond& pc, const float* B, int t, double* X, const mfgp_cg_opts& o,
            mfgp_cg_info* info, double* coeff, int max_iter, const CgBufs& b, const PcgBufs& pb, hipStream_t s) {
    const int64_t n = op.n;
    const int64_t nt = n * t;
    const double tol = o.tol;
    const int max_refine = o.max_refine >= 0 ? o.max_refine : 8;
    int check_every = o.check_every;
    if (check_every <= 0) {
        const double work = static_cast<double>(n) * static_cast<double>(n) * t;
        check_every = work >= 1e9 ? 2 : (work >= 1e8 ? 4 : 8);
    }
    CgState st = make_state(b, X, t, coeff);
    Operator opg;
    GramPrep gpre;
    CG_CHECK(solve_operator(op, b, opg, gpre, s));
    double* rzn = b.scal + 5 * t;     // [t] new r^T z
    double* rrn = b.scal + 6 * t;     // [t] new r^T r (st.rrn holds the current one)
    int* restart = b.ints + 4 * t;

    CG_CHECK(col_dots_ff(B, B, n, t, st.bnorm2, b.dots, s));
    // x = 0, r = b, z = P^-1 r, p = z (the first direction is z itself for
    // every column); keep_iters on a cold restart after a form switch
    auto cold_start = [&](int keep_iters) -> hipError_t {
        hipError_t e = fill_f64(X, nt, 0.0, s);
        if (e == hipSuccess) e = copy2_f32(B, st.r, st.r, nt, s);
        if (e == hipSuccess) e = pc_apply(pc, st.r, t, pb.Zv, pb.pc, s);
        if (e == hipSuccess) e = col_dots_ff(st.r, pb.Zv, n, t, st.rr, b.dots, s);
        if (e == hipSuccess) e = col_dots_ff(st.r, st.r, n, t, rrn, b.dots, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(pcg_init_kernel, dim3(1), dim3(256), 0, s, st, t, tol * tol, rrn, pb.rz0, keep_iters);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        return hipMemcpyAsync(st.p, pb.Zv, nt * sizeof(float), hipMemcpyDeviceToDevice, s);
    };
    CG_CHECK(cold_start(0));

    std::vector<int> h_active(t), h_iters(t), h_status(t), h_restart(t), h_refine(t, 0), h_lan(t);
    std::vector<double> h_relt(t), h_rr(t), h_b2(t);
    // stagnation and precision fallback, as in cg_run (stall.hpp)
    std::vector<StallTracker> h_stall(t);
    std::vector<double> h_t0(t, 1.0);
    std::vector<int> h_nstall(t, 0), h_gaveup(t, 0), h_stalled(t, 0);
    int precision = o.precision;
    int log_coeffs = coeff ? 1 : 0;
    CG_CHECK(hipMemcpyAsync(h_b2.data(), st.bnorm2, t * sizeof(double), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipMemcpyAsync(h_rr.data(), st.rrn, t * sizeof(double), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipStreamSynchronize(s));
    for (int c = 0; c < t; ++c) {
        h_stall[c].begin(0, h_rr[c]);
        if (h_b2[c] > 0.0) h_t0[c] = std::sqrt(h_rr[c] / h_b2[c]);
    }
    const int report_every = o.progress_every > 0 ? o.progress_every : 100;
    int next_report = report_every;
    int steps = 0;   // iterations run by the solver (every cycle; all columns advance together)

    for (;;) {
        CG_CHECK(hipMemcpyAsync(h_active.data(), st.active, t * sizeof(int), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipMemcpyAsync(h_iters.data(), st.iters, t * sizeof(int), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipMemcpyAsync(h_rr.data(), st.rrn, t * sizeof(double), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipStreamSynchronize(s));
        const bool has_next = !op.ski && more_accurate_precision(precision) >= 0;
        bool stop = false;
        for (int c = 0; c < t; ++c) {
            if (!h_active[c] || h_iters[c] >= max_iter) continue;
            if (h_stall[c].update(h_iters[c], h_rr[c])) {
                h_active[c] = 0;
                h_nstall[c] += 1;
                h_stalled[c] = 1;
                stop = true;
            }
        }
        if (stop && has_next) std::fill(h_active.begin(), h_active.end(), 0);   // as in cg_run
        if (stop)
            CG_CHECK(hipMemcpyAsync(st.active, h_active.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
        bool any = false;
        for (int c = 0; c < t; ++c) any = any || (h_active[c] && h_iters[c] < max_iter);
        if (o.progress && steps >= next_report) {
            o.progress(o.progress_user, steps, worst_recurrence(h_active, h_rr, h_b2));
            while (next_report <= steps) next_report += report_every;
        }
        if (any) {
            steps += check_every;
            for (int k = 0; k < check_every; ++k) {
                CG_CHECK(apply_op(opg, st.p, t, st.ap, precision, b, s));
                CG_CHECK(cg_pap_alpha(st, n, t, b.dots, s));
                CG_CHECK(cg_update_rr(st, n, t, b.dots, rrn, s));
                CG_CHECK(pc_apply(pc, st.r, t, pb.Zv, pb.pc, s));
                CG_CHECK(col_dots_ff(st.r, pb.Zv, n, t, rzn, b.dots, s));
                hipLaunchKernelGGL(pcg_beta_kernel, dim3(1), dim3(256), 0, s, st, t, rzn, rrn, tol * tol,
                                   log_coeffs, max_iter);
                hipLaunchKernelGGL(pcg_p_kernel, dim3(nblk(nt)), dim3(256), 0, s, st, pb.Zv, nt, t, nullptr);
                CG_CHECK(hipGetLastError());
            }
            continue;
        }
        // Every column stopped: recompute the true residual in FP64 and refine.
        double* tmp = rzn;
        CG_CHECK(residual_sum(op, B, X, t, b.R64, b.resid, b.sum, s));
        CG_CHECK(col_dots_dd(b.R64, b.R64, n, t, tmp, b.dots, s));
        CG_CHECK(hipMemcpyAsync(h_relt.data(), tmp, t * sizeof(double), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipMemcpyAsync(h_status.data(), st.status, t * sizeof(int), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipStreamSynchronize(s));
        bool again = false, fallback = false;
        const int next_form = op.ski ? -1 : more_accurate_precision(precision);
        bool revive = false;
        for (int c = 0; c < t; ++c) {
            h_relt[c] = h_b2[c] > 0.0 ? std::sqrt(h_relt[c] / h_b2[c]) : 0.0;
            // p^T K_y p <= 0 cannot happen for the SPD K_y: a breakdown with a
            // finite iterate comes from an inexact product form, and the
            // next more accurate form continues from that iterate
            if (h_status[c] == MFGP_BREAKDOWN && next_form >= 0 && std::isfinite(h_relt[c]) &&
                !(h_relt[c] <= tol) && h_refine[c] < max_refine && h_iters[c] < max_iter) {
                h_status[c] = MFGP_OK;
                fallback = revive = true;
            }
            bool need = h_status[c] == MFGP_OK && !(h_relt[c] <= tol) && std::isfinite(h_relt[c]) &&
                        h_refine[c] < max_refine && h_iters[c] < max_iter && !h_gaveup[c];
            if (need && next_form >= 0 && cycle_wants_fallback(h_stalled[c], h_t0[c], h_relt[c], tol)) fallback = true;
            if (need && next_form < 0 && cycle_gave_nothing(h_t0[c], h_relt[c])) {
                h_gaveup[c] = 1;     // the last form cannot improve this column
                need = false;
            }
            h_restart[c] = need ? 1 : 0;
            if (need) {
                h_refine[c] += 1;
                again = true;
            }
        }
        if (!again) break;
        if (fallback) precision = next_form;
        if (fallback && coeff) {
            // as in cg_run: the tridiagonal is recorded anew on the new form
            CG_CHECK(cold_start(1));
            CG_CHECK(hipMemcpyAsync(h_rr.data(), rrn, t * sizeof(double), hipMemcpyDeviceToHost, s));
            CG_CHECK(hipStreamSynchronize(s));
            for (int c = 0; c < t; ++c) {
                h_refine[c] += h_restart[c] ? 0 : 1;   // every column restarts
                h_stall[c].begin(h_iters[c], h_rr[c]);
                h_t0[c] = h_b2[c] > 0.0 ? std::sqrt(h_rr[c] / h_b2[c]) : 1.0;
                h_stalled[c] = 0;
                h_gaveup[c] = 0;
            }
            log_coeffs = 1;
            continue;
        }
        if (revive)
            CG_CHECK(hipMemcpyAsync(st.status, h_status.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
        CG_CHECK(hipMemcpyAsync(restart, h_restart.data(), t * sizeof(int), hipMemcpyHostToDevice, s));
        CG_CHECK(cg_restart(st, b.R64, n, t, restart, s));            // r = fl32(R64) (and p = r)
        CG_CHECK(pc_apply(pc, st.r, t, pb.Zv, pb.pc, s));
        hipLaunchKernelGGL(pcg_p_kernel, dim3(nblk(nt)), dim3(256), 0, s, st, pb.Zv, nt, t, restart);
        CG_CHECK(col_dots_ff(st.r, pb.Zv, n, t, rzn, b.dots, s));
        CG_CHECK(col_dots_ff(st.r, st.r, n, t, rrn, b.dots, s));
        hipLaunchKernelGGL(pcg_activate_kernel, dim3(1), dim3(256), 0, s, st, t, restart, rzn, rrn);
        CG_CHECK(hipGetLastError());
        CG_CHECK(hipMemcpyAsync(h_rr.data(), rrn, t * sizeof(double), hipMemcpyDeviceToHost, s));
        CG_CHECK(hipStreamSynchronize(s));
        for (int c = 0; c < t; ++c) {
            if (!h_restart[c]) continue;
            h_stall[c].begin(h_iters[c], h_rr[c]);
            h_t0[c] = h_relt[c];
            h_stalled[c] = 0;
        }
        log_coeffs = 0;  // the Lanczos tridiagonal belongs to the first cycle only
    }

    CG_CHECK(hipMemcpyAsync(h_rr.data(), st.rrn, t * sizeof(double), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipMemcpyAsync(h_lan.data(), st.lanlen, t * sizeof(int), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipMemcpyAsync(h_iters.data(), st.iters, t * sizeof(int), hipMemcpyDeviceToHost, s));
    CG_CHECK(hipStreamSynchronize(s));
    int worst = MFGP_OK;
    for (int c = 0; c < t; ++c) {
        int stc = h_status[c];
        if (stc == MFGP_OK && !(h_relt[c] <= tol)) stc = MFGP_NOT_CONVERGED;
        if (stc == MFGP_BREAKDOWN)
            worst = MFGP_BREAKDOWN;
        else if (stc == MFGP_NOT_CONVERGED && worst == MFGP_OK)
            worst = MFGP_NOT_CONVERGED;
        if (info) {
            info[c].iters = h_iters[c];
            info[c].lanczos_len = h_lan[c];
            info[c].refinements = h_refine[c];
            info[c].status = stc;
            info[c].rel_resid_recurrence = h_b2[c] > 0.0 ? std::sqrt(h_rr[c] / h_b2[c]) : 0.0;
            info[c].rel_resid_true = h_relt[c];
            info[c].replacements = 0;
            info[c].drift_skips = 0;
            info[c].stalls = h_nstall[c];
            info[c].precision = precision;
        }
    }
    return worst;
}

// Destroys the calling thread's capture streams, each with its device current.
hipError_t release_cg_streams() {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    for (auto& kv : cap_streams) {
        if (hipSetDevice(kv.first) == hipSuccess) (void)hipStreamDestroy(kv.second);
    }
    cap_streams.clear();
    return hipSetDevice(cur);
}

}  // namespace mfgp
