/*
 * mfgp.h -- C ABI of the matrix-free Gaussian-process library for AMD MI355X (gfx950).
 *
 * The library computes, without ever storing the N x N kernel matrix,
 *   K_y V = k(X, X) V + sigma^2 V                       (LightGP Sec. 2, "CG-based inference":
 *                                                          the product CG needs; Sec. 4.1 Table 3)
 * and the conjugate-gradient GP solve built on it: solve, predictive mean,
 * log marginal likelihood and its gradient (Sec. 2, the predictive mean and
 * log p(y|X) formulas; Sec. 3 "Inference": CG with a stochastic Lanczos
 * log-determinant).
 *
 * Conventions shared by every call
 * --------------------------------
 * Layout     X is [n, d] row-major float32.  Right-hand-side blocks (V, B, Z, A)
 *            are [n, t] row-major: column c of row j is element j*t + c.
 * Memory     Every array argument is caller-owned DEVICE memory unless marked
 *            "host".  The library never allocates: scratch comes from the
 *            caller's workspace `ws` of `ws_bytes` bytes (size it with
 *            mfgp_workspace_bytes; 256-byte alignment is handled inside).  No
 *            pointer is kept after a call returns.  Exceptions, cached per
 *            host thread and device on first use: the preconditioned calls'
 *            rocBLAS handle (see "preconditioning"), the hipFFT plans of the
 *            structured-interpolation calls, one per transform shape, whose
 *            tables and work areas hipFFT allocates in device memory, and
 *            the capture stream of the graph-replayed CG iterations (see
 *            mfgp_cg_opts.no_graph; the graphs themselves live for one call);
 *            mfgp_release_thread_resources() frees them.
 * Streams    `stream` is a hipStream_t (NULL = the default stream).  Calls
 *            that return only device results are asynchronous on it; calls
 *            that return host values synchronise it before returning.
 * Errors     Every call returns an mfgp_status.  Argument errors are detected
 *            on the host before anything is launched and leave the outputs
 *            untouched.  No exception crosses the ABI.  MFGP_ERR_HIP carries
 *            the HIP error code in mfgp_last_hip_error() (thread-local).
 * Kernels    family RBF:         k = s2 exp(-r^2 / 2)
 *                   MATERN12:    k = s2 exp(-rho)
 *                   MATERN32:    k = s2 (1 + sqrt3 rho) exp(-sqrt3 rho)
 *                   MATERN52:    k = s2 (1 + sqrt5 rho + 5 rho^2 / 3) exp(-sqrt5 rho)
 *                   PERIODIC:    k = s2 exp(-sum_k 2 sin^2(pi (x_k - x'_k) / p) / l_k^2)
 *                   LINEAR:      k = s2 sum_k x_k x'_k
 *            with r^2 = sum_k ((x_k - x'_k) / l_k)^2, rho = sqrt(r^2), one
 *            lengthscale per dimension when `ard` is set and lengthscale[0]
 *            for all dimensions otherwise, and one period p (the families of
 *            Sec. 3 "Kernels"; s2 is the Scale variance, sigma^2 the noise
 *            variance of Sec. 2).  PERIODIC is evaluated as RBF with unit
 *            lengthscales on the 2d features (cos 2 pi x_k / p, sin 2 pi x_k / p) / l_k,
 *            whose squared distance is sum_k 4 sin^2(pi (x_k - x'_k) / p) / l_k^2;
 *            every product form of RBF applies to it.
 * Sums       (the `+` of Sec. 3 "Kernels"): a kernel whose `next` is non-NULL
 *            is the sum of the chain's terms k = sum_t s2_t k_t(x, x'), at most
 *            MFGP_MAX_TERMS of them, each with its own family, lengthscales,
 *            period and s2 (the `Scale` of each term), all with the head's d;
 *            sigma^2 is the head's noise (the other terms' noise is ignored).
 *            Each term runs its own product form; the terms after the first
 *            add into the result.  Not offered by the batched or preconditioned
 *            calls.  LINEAR terms are rank-d products s2 X (X^T V) with FP64
 *            sums.
 * Products   (the `*` of Sec. 3): a term whose `times` is non-NULL is the
 *            product s2 prod_f k_f of the factor chain (that struct, then its
 *            `times` chain), s2 being the first factor's outputscale (the
 *            other factors' outputscale, noise and `next` are ignored).
 *            Factors are RBF or PERIODIC (at most one PERIODIC), at most
 *            MFGP_MAX_TERMS of them, each with the head's d and with at most
 *            MFGP_MAX_D features in all (d per RBF factor, 2d for the
 *            periodic one): such a product is RBF with unit lengthscales on
 *            the concatenated features and runs every RBF product form.
 *            Other factor families return MFGP_UNSUPPORTED.
 * Gradients  are with respect to the positive parameters in the order
 *            [l_1 .. l_d] (ard) or [l] (shared), then p (PERIODIC only), then
 *            s2 (LINEAR: s2 only), then sigma^2; for a product term, every
 *            factor's lengthscales (and p) in factor order, then s2; for a
 *            sum, every term's parameters without sigma^2 in chain order,
 *            then sigma^2 (mfgp_num_params of them).
 * Feature dimension  the d argument of the workspace-size queries is the
 *            kernel's feature dimension mfgp_feature_dim(kern): the input
 *            dimension, twice it for PERIODIC, summed over a sum's terms.
 * Threads    The library is reentrant: no mutable globals besides the
 *            thread-local last HIP error, the thread-local rocBLAS handles
 *            and hipFFT plans (see Memory), and the per-device address of the
 *            fixed workspace of mfgp_kernel_matvec_noalloc (set once, under a
 *            lock).  The MLL calls compute the stochastic Lanczos quadratures
 *            on short-lived host threads of their own (at most 16 for a
 *            batch, started and joined within the call; the batched call runs
 *            a problem's quadratures while the other problems iterate).
 */
#ifndef MFGP_H
#define MFGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFGP_MAX_D 8
#define MFGP_MAX_T 64
#define MFGP_MAX_RANK 1024   /* largest pivoted-Cholesky preconditioner rank */
#define MFGP_MAX_TERMS 4     /* terms of a kernel sum (mfgp_kernel.next chain) */

typedef enum {
    MFGP_RBF = 0,
    MFGP_MATERN12 = 1,
    MFGP_MATERN32 = 2,
    MFGP_MATERN52 = 3,
    MFGP_PERIODIC = 4,    /* d <= MFGP_MAX_D / 2; not offered by the batched calls */
    MFGP_LINEAR = 5       /* k = s2 x.x'; no lengthscale; not offered by the batched
                             or preconditioned calls                               */
} mfgp_family;

/* Arithmetic of the product (kernel entries are always float32).  The
 * FP32-class forms (0, 3, 5, 6) are held to the FP32 bar (per-column
 * relative error <= 1e-5 against FP64); the bf16 forms are described below. */
typedef enum {
    MFGP_FP32 = 0,    /* FP32, fastest form that applies:
                         - square products of RBF-class terms (RBF, PERIODIC,
                           their products; a two-term sum of them as one fused
                           sweep) with n >= 32768 and t = 1 or
                           16 k + {0, 1} (k = 1..4): squared distances from the
                           Gram form |g_i|^2 + |g_j|^2 - 2 g_i.g_j on FP32 MFMA
                           (g = prescaled points minus their mean), checked on
                           the device: where max |g|^2 > 64 the launch uses
                           direct differences instead (the form's error grows
                           with |g|^2);
                         - else, for t = 16 k + {0, 1}: direct differences, the
                           16-column tiles of the contraction on FP32 MFMA
                           (v_mfma_f32_16x16x4_f32);
                         - else the vector ALU (MFGP_FP32_VALU).             */
    MFGP_BF16X1 = 1,  /* entries and V rounded to bf16, MFMA, FP32 accumulation    */
    MFGP_BF16X2 = 2,  /* bf16 hi/lo split of both operands (3 MFMA products)        */
    MFGP_FP32_VALU = 3, /* FP32 direct differences, contraction on the vector ALU   */
    MFGP_BF16X3 = 4,  /* exact three-way bf16 split of both operands, 6 of the 9
                          MFMA products (the dropped ones are < 2^-23 |K V|):
                          binary32-class products on the bf16 matrix cores        */
    MFGP_FP32_DIRECT = 5, /* MFGP_FP32 without the Gram form                       */
    MFGP_FP32_GRAM = 6    /* MFGP_FP32 with the Gram form at any n (square RBF
                             products; otherwise as MFGP_FP32_DIRECT).  Not
                             offered by the batched calls (MFGP_UNSUPPORTED).   */
} mfgp_precision;
/* The bf16 forms take t <= 65 columns; for t = 32 k + 1 column 0 (y of a
 * [y, probes] block) is contracted on the vector ALU in FP32. */

typedef enum {
    MFGP_OK = 0,
    MFGP_ERR_ARG = 1,          /* invalid argument, detected before any launch       */
    MFGP_ERR_HIP = 2,          /* a HIP runtime call failed, see mfgp_last_hip_error */
    MFGP_ERR_WORKSPACE = 3,    /* ws_bytes below mfgp_workspace_bytes(...)           */
    MFGP_NOT_CONVERGED = 4,    /* CG stopped at max_iter / max_refine; best iterate written */
    MFGP_BREAKDOWN = 5,        /* p^T K_y p <= 0 or non-finite; best iterate written  */
    MFGP_UNSUPPORTED = 6       /* valid but not provided (e.g. d > MFGP_MAX_D)        */
} mfgp_status;

/* Workspace query operation codes. */
typedef enum {
    MFGP_OP_MATVEC = 0,
    MFGP_OP_CG = 1,
    MFGP_OP_PREDICT = 2,
    MFGP_OP_MLL = 3,
    MFGP_OP_ADJOINT = 4,
    MFGP_OP_RESIDUAL = 5,
    MFGP_OP_PCHOL = 6,     /* mfgp_pivoted_cholesky (mfgp_precond_workspace_bytes)  */
    MFGP_OP_PAPPLY = 7,    /* mfgp_precond_apply                                     */
    MFGP_OP_PCG = 8,       /* mfgp_precond_cg_solve                                  */
    MFGP_OP_PMLL = 9       /* mfgp_precond_mll_and_grad                              */
} mfgp_op;

/* Kernel hyperparameters (host struct, passed by pointer). */
typedef struct mfgp_kernel_s {
    int32_t family;                       /* mfgp_family                               */
    int32_t d;                            /* input dimension, 1..MFGP_MAX_D             */
    int32_t ard;                          /* nonzero: one lengthscale per dimension     */
    float lengthscale[MFGP_MAX_D];        /* > 0, finite; [0] only when ard == 0        */
    float outputscale;                    /* s2 > 0                                     */
    float noise;                          /* sigma^2 >= 0 (> 0 for solves)              */
    float period;                         /* PERIODIC: p > 0, finite; ignored otherwise  */
    const struct mfgp_kernel_s* next;     /* host: next term of a sum, or NULL          */
    const struct mfgp_kernel_s* times;    /* host: next factor of a product, or NULL    */
} mfgp_kernel;

/* Conjugate-gradient options (host struct). */
typedef struct {
    double tol;           /* per column ||b - K_y x||_2 / ||b||_2 target, > 0 (e.g. 1e-6)      */
    int32_t max_iter;     /* CG iterations per column over all refinement cycles;
                             0 = min(max(2n, 64), 20000)                                   */
    int32_t check_every;  /* iterations between host convergence checks; 0 = automatic       */
    int32_t max_refine;   /* residual recomputations / restarts allowed; < 0 = default 8      */
    int32_t precision;    /* mfgp_precision of the CG matvec (residuals always FP32 entries from
                             direct differences, FP64 sums) */
    int32_t warm_start;   /* nonzero: Xsol holds the initial guess x0 on entry                */
    int32_t no_replacement; /* nonzero: no residual replacement while iterating (restarts
                             from the recomputed residual after each cycle only).  Even
                             when zero, replacement runs only if the host checks at
                             least every other iteration (check_every <= 2; automatic
                             for products of >= 1e9 entry-columns)                      */
    uint64_t probe_seed;  /* seed of the SplitMix64 probes when Z == NULL (mll_and_grad)      */
    /* Optional progress callback (may be NULL), called from the calling thread
     * at host convergence checks whenever the solver has run progress_every
     * (0 = 100) more iterations since the last call: progress(progress_user,
     * iterations run so far (every cycle; all columns advance together), the
     * worst ||r||/||b|| of the recurrence over the columns still iterating). */
    void (*progress)(void* user, int32_t iterations, double rel_resid);
    void* progress_user;
    int32_t progress_every;
    int32_t no_graph;     /* nonzero: launch every iteration's kernels directly.  Otherwise,
                             when the host checks every 4 or more iterations (automatic for
                             products of < 1e9 entry-columns) and the operator is not SKI,
                             the iterations between checks are captured once into a HIP
                             graph (on a capture stream cached per host thread, see
                             mfgp_release_thread_resources) and replayed on `stream`: the
                             same kernels with the same arguments, so the same results */
} mfgp_cg_opts;

/* Per-column CG report (host array, one entry per column). */
typedef struct {
    int32_t iters;                /* CG iterations performed (all cycles)                   */
    int32_t lanczos_len;          /* iterations of the first cycle (SLQ length m)           */
    int32_t refinements;          /* restarts: from a recomputed residual, or from x = 0
                                     when the product form switches while the Lanczos
                                     tridiagonal is recorded (the SLQ then describes the
                                     form the solution converges on)                     */
    int32_t status;               /* mfgp_status of this column                             */
    double rel_resid_recurrence;  /* ||r_k||/||b|| carried by the recurrence at exit        */
    double rel_resid_true;        /* recomputed ||b - K_y x||/||b||, K_y with FP32 entries,
                                     FP64 accumulation, x in FP64                          */
    int32_t replacements;         /* residual replacements applied (small drift only)       */
    int32_t drift_skips;          /* replacements refused because the recurrence had
                                     drifted more than 10% from the true residual           */
    int32_t stalls;               /* cycles ended early: by stagnation (after falling
                                     tenfold, the recurrence residual made no new minimum
                                     for max(100, cycle length / 4) iterations), or by a
                                     replacement that found the recurrence drifted away
                                     from a true residual still far above tol            */
    int32_t precision;            /* mfgp_precision of the products of the last cycle: the
                                     requested one, or a more accurate form taken after a
                                     cycle that ended early, cut the true residual by less
                                     than 0.7x, or ended where two more cycles of the same
                                     reduction would stay above tol (x1 -> x2 -> x3 ->
                                     MFGP_FP32_DIRECT; the batched solver keeps its form) */
} mfgp_cg_info;

/* Feature dimension of a kernel (the d of the workspace-size queries): kern->d,
 * 2 kern->d for MFGP_PERIODIC, summed over the terms of a sum; 0 for a NULL
 * kernel or kern->d < 1. */
int mfgp_feature_dim(const mfgp_kernel* kern);

/* Bytes of workspace a call needs.  op: mfgp_op; n rows; d = mfgp_feature_dim; t columns
 * (matvec/cg/adjoint/residual), test points m for MFGP_OP_PREDICT passed in t
 * as the column count of alpha and in max_iter as m; number of probes + 1 for
 * MFGP_OP_MLL; max_iter as passed in mfgp_cg_opts (0 = default).  Returns 0 for
 * invalid sizes. */
size_t mfgp_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t t, int32_t precision,
                            int32_t max_iter);

/* KV = K_y V = s2 k(X, X) V + sigma^2 V  (Sec. 2; Sec. 4.1 Table 3, the fused
 * matrix-free product).  X [n,d], V [n,t], KV [n,t] (must not alias V).
 * precision: mfgp_precision.  Asynchronous. */
int mfgp_kernel_matvec(const mfgp_kernel* kern, const float* X, int64_t n, const float* V,
                       int32_t t, float* KV, int32_t precision, void* ws, size_t ws_bytes,
                       void* stream);

/* Capacity of the fixed device workspace of mfgp_kernel_matvec_noalloc (bytes). */
#define MFGP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* mfgp_kernel_matvec without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * mfgp_kernel_matvec; the scratch is a fixed device array of
 * MFGP_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends.  The call allocates nothing (no hipMalloc / hipFree, no
 * allocating library routine).
 * Limit: returns MFGP_ERR_WORKSPACE, launching nothing, when
 * mfgp_workspace_bytes(MFGP_OP_MATVEC, n, mfgp_feature_dim(kern), t,
 * precision, 0) exceeds MFGP_NOALLOC_SCRATCH_BYTES (e.g. n = 1e5, d = 4 fits
 * for t <= 8).  `stream` must belong to the current device (MFGP_ERR_ARG
 * otherwise).  The first call on a device looks up that device's array.
 * Every call on one GPU shares its array: calls that overlap in time on one
 * GPU (two streams, or two threads) race and give undefined results; calls
 * on one stream are ordered and safe.  Each call writes every scratch value
 * it reads, so nothing carries over between calls.  Asynchronous. */
int mfgp_kernel_matvec_noalloc(const mfgp_kernel* kern, const float* X, int64_t n, const float* V,
                               int32_t t, float* KV, int32_t precision, void* stream);

/* R = B - K_y Xsol with the library's FP32 kernel entries accumulated in FP64
 * (the recomputed residual of the solver).  B [n,t] float32, Xsol [n,t]
 * float64, R [n,t] float64 (device).  rel (host, optional, [t]) receives
 * ||R_c||_2 / ||B_c||_2; when rel is non-NULL the call synchronises. */
int mfgp_residual(const mfgp_kernel* kern, const float* X, int64_t n, const float* B,
                  const double* Xsol, int32_t t, double* R, double* rel, void* ws,
                  size_t ws_bytes, void* stream);

/* Solve K_y Xsol = B column by column with unpreconditioned conjugate
 * gradients (Sec. 2 "CG-based inference"; Sec. 5: the plain CG loop), started
 * at x0 = 0 (or at Xsol when opts->warm_start), FP32 vectors and FP64 scalars,
 * with the true residual recomputed (mfgp_residual) once the recurrence meets
 * tol, and restarts from it until it does (iterative refinement).  Columns
 * converge independently and freeze.
 * B [n,t] float32; Xsol [n,t] float64 (in: x0 if warm_start, out: solution).
 * info: host [t].  lanczos: optional device [t][max_iter][2] float64 receiving
 * (alpha_j, beta_j) of each column's first cycle (the stochastic-Lanczos input);
 * entries past info[c].lanczos_len are unspecified.  Synchronises.  Returns
 * the worst column status. */
int mfgp_cg_solve(const mfgp_kernel* kern, const float* X, int64_t n, const float* B,
                  int32_t t, double* Xsol, const mfgp_cg_opts* opts, mfgp_cg_info* info,
                  double* lanczos, void* ws, size_t ws_bytes, void* stream);

/* MU = s2 k(Xs, X) A  (Sec. 2: mu_* = K_*f (K_ff + sigma^2 I)^{-1} y with
 * A = the solve's result).  Xs [m,d], A [n,t] float32, MU [m,t].  No noise
 * term.  Asynchronous. */
int mfgp_predict_mean(const mfgp_kernel* kern, const float* X, int64_t n, const float* Xs,
                      int64_t m, const float* A, int32_t t, float* MU, void* ws,
                      size_t ws_bytes, void* stream);

/* Stochastic Lanczos quadrature of one probe from its CG coefficients
 * (host only, no GPU): with T the Lanczos tridiagonal that the coefficients
 * define (T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_j,j+1 = sqrt(beta_j)/alpha_j),
 * *q = znorm2 * e_1^T log(T) e_1.  coeffs: host [m][2] (alpha_j, beta_j). */
int mfgp_slq_quadrature(const double* coeffs, int32_t m, double znorm2, double* q);

/* Log marginal likelihood and gradient (Sec. 2: log p(y|X) =
 * -1/2 [y^T K_y^{-1} y + log|K_y| + N log 2 pi]; Sec. 3: CG with a stochastic
 * Lanczos log-determinant; Sec. 4.3: Rademacher probes).
 * One batched CG solve of [y, Z] (t = num_probes + 1 columns) gives
 * alpha = K_y^{-1} y, U = K_y^{-1} Z and per-probe Lanczos coefficients;
 * log|K_y| ~= (1/p) sum_c ||z_c||^2 e_1^T log(T_c) e_1; the gradient is
 * 1/2 alpha^T dK alpha - 1/(2p) sum_c u_c^T dK z_c, its lengthscale and
 * outputscale parts from one fused adjoint pass over all kernel entries.
 * y [n]; Z [n,p] (+-1 probes) or NULL to draw them on the device from
 * opts->probe_seed (SplitMix64, see mfgp_rademacher).  Host outputs: mll,
 * logdet (optional), grad (optional, [n_theta]); device output alpha_out
 * (optional, [n] float64); info (optional, host [p+1]).  Synchronises. */
int mfgp_mll_and_grad(const mfgp_kernel* kern, const float* X, int64_t n, const float* y,
                      int32_t num_probes, const float* Z, const mfgp_cg_opts* opts, double* mll,
                      double* logdet, double* grad, double* alpha_out, mfgp_cg_info* info,
                      void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of the operator:
 * grad[theta] = sum_c colw[c] A_c^T (dK_y/dtheta) B_c for every parameter
 * (lengthscales, s2, sigma^2).  A, B [n,t] float32; colw host [t]; grad host
 * [n_theta].  Synchronises. */
int mfgp_kernel_adjoint(const mfgp_kernel* kern, const float* X, int64_t n, const float* A,
                        const float* B, int32_t t, const double* colw, double* grad, void* ws,
                        size_t ws_bytes, void* stream);

/* Z [n,p] float32 Rademacher probes: entry (j, c) is +1 when bit 63 of
 * SplitMix64 output number c*n + j + 1 of the stream seeded with `seed` is
 * clear, else -1 (Steele, Lea & Flood 2014).  Asynchronous. */
int mfgp_rademacher(uint64_t seed, int64_t n, int32_t p, float* Z, void* stream);

/* ---------------------------------------------------------------- structured kernel interpolation
 * SKI / KISS-GP (Sec. 2 "Structured kernel interpolation"; Sec. 3 "Inference":
 * SKI with FFT), the method of Wilson & Nickisch (2015):
 *   K_y V ~ W K_UU W^T V + sigma^2 V,   mu_* ~ W_* K_UU W^T A,   K_UU = s2 k(U, U),
 * U a regular grid (D <= 3), W local cubic convolution interpolation (Keys
 * 1981, a = -1/2; 4^D weights per point), K_UU applied through the FFT (FP64,
 * hipFFT) of its circulant embedding (2 m_k per dimension).  Grid per
 * dimension k: the data range [min_k, max_k] (the points' own, or the
 * caller's when explicit_range is set), r_k = max_k - min_k (1 if zero),
 * spacing h_k = r_k / (m_k - 4), nodes lo_k + j h_k with lo_k = min_k - h_k,
 * j < m_k; weights of nodes off the grid (points outside the range) are
 * dropped.  Products accumulate in FP64 and round once (the points are
 * bucketed by stencil cell with atomic placement, so the order of a cell's
 * terms, and the last bits, may vary between runs).  Kernels: one term of family RBF, MATERN*
 * or PERIODIC (no sums, products or LINEAR: MFGP_UNSUPPORTED), d <= 3.
 * The first call with a grid shape and column count on a device from a host
 * thread creates hipFFT plans for it and keeps them until the process ends
 * (hipFFT allocates their device memory then); later calls reuse them. */
typedef struct {
    int32_t m[3];            /* grid nodes per dimension (first d used), >= 5;
                                prod (2 m_k) < 2^31                                 */
    int32_t explicit_range;  /* nonzero: lo / hi give the data range                */
    float lo[3];             /* explicit_range: min_k (finite)                      */
    float hi[3];             /* explicit_range: max_k (finite, >= lo[k])            */
} mfgp_ski_grid;

/* Bytes of workspace of a SKI call: op MFGP_OP_MATVEC / MFGP_OP_CG /
 * MFGP_OP_PREDICT / MFGP_OP_MLL (t = probes + 1), n points, d dims, t
 * columns, the grid (host); 0 if invalid. */
size_t mfgp_ski_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t t, const mfgp_ski_grid* grid);

/* KV = W K_UU W^T V + sigma^2 V on the grid of X (or the explicit range).
 * X [n,d], V [n,t], KV [n,t] (must not alias V).  Asynchronous. */
int mfgp_ski_matvec(const mfgp_kernel* kern, const float* X, int64_t n, const mfgp_ski_grid* grid,
                    const float* V, int32_t t, float* KV, void* ws, size_t ws_bytes, void* stream);

/* Solve (W K_UU W^T + sigma^2 I) Xsol = B by the CG of mfgp_cg_solve (same
 * options, refinement against the FP64 SKI residual; opts->precision is not
 * used: the SKI product is FP64).  Synchronises. */
int mfgp_ski_cg_solve(const mfgp_kernel* kern, const float* X, int64_t n, const mfgp_ski_grid* grid,
                      const float* B, int32_t t, double* Xsol, const mfgp_cg_opts* opts, mfgp_cg_info* info,
                      void* ws, size_t ws_bytes, void* stream);

/* MU = W_* K_UU W^T A: the SKI predictive mean at Xs [m,d] from A [n,t]
 * (the solve's result), on the grid of X and Xs together (or the explicit
 * range; use the same grid as the solve).  Asynchronous. */
int mfgp_ski_predict_mean(const mfgp_kernel* kern, const float* X, int64_t n, const float* Xs, int64_t m,
                          const mfgp_ski_grid* grid, const float* A, int32_t t, float* MU, void* ws,
                          size_t ws_bytes, void* stream);

/* Log marginal likelihood of the SKI model and its gradient: as
 * mfgp_mll_and_grad with K_ff replaced by W K_UU W^T on the grid (CG on the
 * SKI operator, stochastic Lanczos log-determinant over the probes, the
 * gradient 1/2 a^T dK a - 1/(2p) sum_c u_c^T dK z_c with dK = W (dK_UU) W^T:
 * one spectral product of W^T [a, Z] per parameter).  num_probes + 1 <=
 * MFGP_MAX_T; opts->max_iter must be 0 (the default cap, which the workspace
 * query MFGP_OP_MLL with t = num_probes + 1 assumes).  Synchronises. */
int mfgp_ski_mll_and_grad(const mfgp_kernel* kern, const float* X, int64_t n, const mfgp_ski_grid* grid,
                          const float* y, int32_t num_probes, const float* Z, const mfgp_cg_opts* opts, double* mll,
                          double* logdet, double* grad, mfgp_cg_info* info, void* ws, size_t ws_bytes,
                          void* stream);

/* ---------------------------------------------------------------- batches
 * Many independent GP problems solved together (LightGP Sec. 5 names batched
 * solves as the missing piece of its CG).  Problem b has n[b] rows, its own
 * input dimension kern[b].d and hyperparameters kern[b] (all problems share
 * kern[0].family).  Packed layouts (device, caller-owned):
 *   X   problem b's [n_b, d_b] row-major block starts at element x_off[b];
 *   y   [sum n_b] float32, problem b's rows start at row_off[b];
 *   Z   [sum n_b, p] float32 probes (rows as y), or NULL for SplitMix64
 *       probes drawn per problem from probe_seed + b.
 * The sweeps of all problems run in ONE persistent launch per product: a
 * work queue of (problem, 256-row block, j-range) tiles in longest-first
 * order, pulled by resident workgroups through an atomic counter.  The CG
 * iterations of the batch are captured into a hipGraph and replayed between
 * host convergence checks.  The j-range length of the tiles is chosen by the
 * plan's autotuner (timed on the first call when tuning is enabled). */
typedef struct {
    int32_t nprob;
    const int64_t* n;          /* host [nprob] rows per problem                 */
    const int64_t* row_off;    /* host [nprob] first row of problem b in y / Z  */
    const int64_t* x_off;      /* host [nprob] element offset of X_b in X       */
    const mfgp_kernel* kern;   /* host [nprob]                                  */
} mfgp_batch;

/* Opaque batch plan: host copies of the batch description, the tile queue,
 * the tuned tile length and the captured CG graph.  The only object in the
 * library that keeps state between calls; it owns no device memory. */
typedef struct mfgp_batch_plan_s* mfgp_batch_plan;

/* Creates a plan for batches of this shape with p = num_probes probes
 * (t = p + 1 columns, which must be one of 1..8, 16, 17, 32, 33).  tune: 1 =
 * time the candidate tile lengths on the first mfgp_batch_mll_and_grad call,
 * 0 = use the built-in default.  use_graph: capture CG iterations.  max_iter 0
 * selects min(max(2 max_b n_b, 64), 20000).  Host only: it validates before
 * touching the device.  Errors: MFGP_ERR_ARG for a NULL pointer, nprob < 1,
 * num_probes < 1, max_iter < 0, n_b < 1, d_b outside 1..MFGP_MAX_D, a family
 * differing from kern[0].family, a non-finite or non-positive lengthscale,
 * outputscale or noise, a negative offset, or row_off that is not the prefix
 * sum of n (rows must be packed back to back in problem order);
 * MFGP_UNSUPPORTED for a column count without a compiled kernel, the
 * MFGP_PERIODIC or MFGP_LINEAR family, a kernel sum or product (next or
 * times != NULL), or a problem with n_b > 2^24 rows (the per-problem fragment
 * indices are 32-bit). */
int mfgp_batch_plan_create(const mfgp_batch* batch, int32_t num_probes, int32_t max_iter,
                           int32_t tune, int32_t use_graph, mfgp_batch_plan* plan);
int mfgp_batch_plan_destroy(mfgp_batch_plan plan);
/* Workspace bytes of mfgp_batch_mll_and_grad for this plan. */
size_t mfgp_batch_workspace_bytes(mfgp_batch_plan plan);
/* Tile length in use (0 before tuning), its measured sweep time and the
 * number of graph replays of the last call (host outputs, may be NULL). */
int mfgp_batch_plan_info(mfgp_batch_plan plan, int64_t* tile_j, double* tuned_sweep_ms,
                         int64_t* graph_launches);

/* For every problem b: log marginal likelihood, stochastic Lanczos log-det and
 * gradient exactly as mfgp_mll_and_grad defines them, computed for the whole
 * batch at once.  Host outputs: mll [nprob], logdet [nprob] (optional), grad
 * (optional, problem b's n_theta entries packed one problem after another),
 * info (optional, [nprob][p+1]).  opts->precision: MFGP_FP32 (the FP32-MFMA
 * contraction where t = 16 k + {0,1}), MFGP_FP32_VALU, or the bf16 forms
 * MFGP_BF16X1/X2/X3 (tile lengths are re-tuned when the precision changes);
 * opts->progress, if set, reports the iterations run and the worst recurrence
 * residual over the columns of the batch still iterating.  Synchronises.  Returns the
 * worst status over all problems. */
int mfgp_batch_mll_and_grad(mfgp_batch_plan plan, const float* X, const float* y, const float* Z,
                            const mfgp_cg_opts* opts, double* mll, double* logdet, double* grad,
                            mfgp_cg_info* info, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- predictive variance
 * The latent predictive variance diag(Sigma_*) of Sec. 2,
 *   Sigma_* = K_** - K_*f K_y^{-1} K_f*,
 * on the CG path by the stochastic diagonal estimator (Bekas, Kokiopoulou &
 * Saad 2007; the Rademacher-probe estimator of the accuracy section): with
 * probe columns z_c over the m test points and A = K_*f K_y^{-1} K_f*,
 *   var[q] = s2 - sum_c Z[q][c] (A Z)[q][c] / sum_c Z[q][c]^2.
 * A Z is two rectangular FP32 sweeps around one CG solve with p right-hand
 * sides (mfgp_cg_solve's solver, stopping rule and refinement).  Unbiased
 * for Rademacher probes; exact for Z = the m x m identity (p = m).  The
 * noise variance of a new observation is not added. */

/* Workspace bytes of mfgp_predict_variance (0 if invalid). */
size_t mfgp_variance_workspace_bytes(int64_t n, int32_t d, int64_t m, int32_t p, int32_t precision);
/* X [n][d] training inputs, Xs [m][d] test inputs, Z [m][p] probes (device;
 * NULL: Rademacher probes from opts->probe_seed, laid out as mfgp_rademacher
 * with n = m).  var [m] (device, float32) receives the estimate; info
 * (optional, host [p]) the CG result per probe column.  Synchronises.
 * Returns the CG status (MFGP_NOT_CONVERGED / MFGP_BREAKDOWN still write
 * var from the best iterate). */
int mfgp_predict_variance(const mfgp_kernel* kern, const float* X, int64_t n, const float* Xs, int64_t m,
                          int32_t p, const float* Z, const mfgp_cg_opts* opts, float* var, mfgp_cg_info* info,
                          void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- preconditioning
 * LightGP's CG is unpreconditioned; Sec. 5 ("Limitations") names the
 * comparison system's pivoted-Cholesky-preconditioned, batched CG as what it
 * lacks.  These calls add that preconditioner (the construction of Gardner et
 * al. 2018 with the greedy pivoted Cholesky of Harbrecht, Peters & Schneider
 * 2012) to the same matrix-free operator:
 *   P = L L^T + sigma^2 I, L the rank-k pivoted Cholesky factor of the
 *   noise-free s2 k(X, X) (entries generated as in the sweeps), applied by the
 *   Woodbury identity (k x k system factored in FP64);
 *   preconditioned CG with the stopping rule, FP64 solution and refinement of
 *   mfgp_cg_solve (no residual replacement);
 *   log|K_y| = log|P| + SLQ of P^{-1/2} K_y P^{-1/2} with probes z ~ N(0, P);
 *   tr(K_y^{-1} dK) ~ (1/p) sum_c (K_y^{-1} z_c)^T dK (P^{-1} z_c).
 * L is a device array [rank][n] float32 (row q holds column q of the factor),
 * caller-owned; it is built by mfgp_pivoted_cholesky and read by the others.
 * Workspace sizes come from mfgp_precond_workspace_bytes.  The kernel calls
 * (pivoted Cholesky, PCG, PMLL) take one stationary, periodic or product
 * term: MFGP_LINEAR and kernel sums return MFGP_UNSUPPORTED.
 * The Woodbury products run as rocBLAS FP64 GEMMs and triangular solves
 * (atomics off: reproducible).  The first call of mfgp_precond_apply,
 * _cg_solve or _mll_and_grad on a device from a host thread creates a rocBLAS
 * handle for that pair and keeps it until the process ends; rocBLAS
 * allocates its own device memory for it then.  Every later call reuses it. */

/* Bytes of workspace of a preconditioned call: op MFGP_OP_PCHOL / PAPPLY /
 * PCG / PMLL; t right-hand sides (probes + 1 for PMLL); rank k <= min(n,
 * MFGP_MAX_RANK); precision and max_iter as in mfgp_cg_opts.  0 if invalid. */
size_t mfgp_precond_workspace_bytes(int32_t op, int64_t n, int32_t d, int32_t t, int32_t rank,
                                    int32_t precision, int32_t max_iter);
/* Rank-k pivoted Cholesky of s2 k(X, X): L [rank][n] and the pivot indices
 * piv [rank] (device outputs).  Greedy pivot = largest remaining diagonal
 * (ties: smallest index); columns past the numerical rank (remaining diagonal
 * <= 1e-6 s2) are zero.  Asynchronous. */
int mfgp_pivoted_cholesky(const mfgp_kernel* kern, const float* X, int64_t n, int32_t rank, float* L,
                          int32_t* piv, void* ws, size_t ws_bytes, void* stream);
/* Probes z_c ~ N(0, P) from standard normal draws: Z = L^T-factor E +
 * sqrt(noise) G, i.e. Z[j][c] = sum_q L[q][j] E[q][c] + sqrt(noise) G[j][c];
 * E [rank][p], G [n][p], Z [n][p] device.  Asynchronous. */
int mfgp_precond_probes(const float* L, int64_t n, int32_t rank, float noise, const float* E,
                        const float* G, int32_t p, float* Z, void* stream);
/* Zout = P^{-1} R for R [n][t] (device); logdet (host, optional) = log|P|.
 * Synchronises (the k x k factorisation runs on the host).  MFGP_BREAKDOWN if
 * sigma^2 I + L^T L is not positive definite. */
int mfgp_precond_apply(const float* L, int64_t n, int32_t rank, float noise, const float* R, int32_t t,
                       float* Zout, double* logdet, void* ws, size_t ws_bytes, void* stream);
/* Preconditioned CG on K_y Xsol = B (as mfgp_cg_solve; opts->warm_start and
 * residual replacement are not used).  lanczos (optional, device
 * [t][max_iter][2]) receives the first cycle's (alpha, beta).  Synchronises. */
int mfgp_precond_cg_solve(const mfgp_kernel* kern, const float* X, int64_t n, const float* B, int32_t t,
                          double* Xsol, const float* L, int32_t rank, const mfgp_cg_opts* opts,
                          mfgp_cg_info* info, double* lanczos, void* ws, size_t ws_bytes, void* stream);
/* Log marginal likelihood and gradient as mfgp_mll_and_grad, with the
 * preconditioned solver and estimators above.  Z [n][p] (device) must be
 * probes drawn from N(0, P) (e.g. by mfgp_precond_probes).  Synchronises. */
int mfgp_precond_mll_and_grad(const mfgp_kernel* kern, const float* X, int64_t n, const float* y,
                              int32_t num_probes, const float* Z, const float* L, int32_t rank,
                              const mfgp_cg_opts* opts, double* mll, double* logdet, double* grad,
                              double* alpha_out, mfgp_cg_info* info, void* ws, size_t ws_bytes,
                              void* stream);

/* Kernel timing (for benchmarks).  While enabled on the calling thread, every
 * entry-sweep launch (the fused K-tile kernels) is bracketed by HIP events
 * recorded on the stream the sweep is launched on, and its algorithmic work
 * is tallied: entries generated and FLOP by the per-entry counts (RBF
 * 3d+1+2t, Matern-1/2 3d+2+2t, Matern-3/2 3d+5+2t, Matern-5/2 3d+7+2t,
 * adjoint 5d+4+2t; exp and sqrt count as one).  Sweep kinds: 0 FP32 sweeps
 * (matvec, CG, predict), 1 FP64-accumulated residual sweeps, 2 adjoint
 * sweeps, 3 BF16-MFMA sweeps; -1 selects all.  mfgp_mll_and_grad also
 * records the host wall time of its phases (CG solve, quadrature, adjoint).
 * mfgp_timing_read synchronises the recorded events and returns totals since
 * the last enable (host outputs, any may be NULL).  Thread-local state. */
int mfgp_timing_enable(int32_t on);
int mfgp_timing_read(int32_t kind, double* sweep_ms, int64_t* launches, double* entries,
                     double* flops);
int mfgp_timing_phases(double* cg_ms, double* slq_ms, double* adjoint_ms);

/* Number of gradient entries for a kernel: (ard ? d : 1) + 2, + 1 for
 * MFGP_PERIODIC, 2 for MFGP_LINEAR; a product term counts its factors'
 * lengthscales and period, s2 and sigma^2; for a sum, the terms' counts less
 * one each, plus one (sigma^2). */
int mfgp_num_params(const mfgp_kernel* kern);

const char* mfgp_status_string(int status);
int mfgp_last_hip_error(void);
int mfgp_version(void);

/* Frees the calling thread's cached library resources on every device: the
 * rocBLAS handles of the preconditioned calls, the hipFFT plans (with their
 * device memory) of the structured-interpolation calls and the CG capture
 * streams.  Later calls
 * create them again.  Call it with no library work of this thread in flight.
 * Returns MFGP_ERR_HIP if switching devices fails. */
int mfgp_release_thread_resources(void);

#ifdef __cplusplus
}
#endif

#endif /* MFGP_H */
