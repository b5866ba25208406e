"""Benchmark: one step = the whole GP hot path on the 100k workload.

Workload (synthetic): N = 100000, d = 4, X ~ U[-1,1]^4, RBF l = 0.3, s^2 = 1,
sigma^2 = 0.01, y = sum_k sin(pi x_k) + N(0, 0.1^2), 32 Rademacher probes.
One step runs, on inputs already resident in HBM:
  mll_and_grad  -- prescale, batched CG on [y, Z] (t = 33) to a recomputed
                   residual <= 1e-6 with refinement, stochastic Lanczos
                   log-determinant, MLL, and the adjoint gradient pass;
  predict_mean  -- mu = K(X*, X) alpha at 2000 test points.
`value` is kernel entries generated per second over the timed steps (every
entry sweep counted once per launch).  The line also carries the CG solve
time, the MLL+grad time, the roofline of the dominant kernel (the FP32
entry sweep, timed live with HIP events on its launch stream), the paper's
Table 3 product (t = 1) on the same points with its own roofline, the same
step in the other product forms (median of --compare-reps runs; the BF16
forms with their VALU-generation and matrix-core contraction rooflines), the
preconditioned step, and the oracle's host throughput on a bounded sample.

python bench.py [--steps K] [--warmup W] [--precision fp32|bf16x1|bf16x2|bf16x3] [--no-cpu-baseline]
python bench.py --mode kernel [--reps R] [--precision P] [--cols T]   (profiling helper: R
    launches of the step's dominant product, K_y V at t = 33 (or the first T columns
    of [y, probes]) in the chosen form, then a 1 GiB device copy whose FETCH_SIZE /
    WRITE_SIZE calibrate the HBM-traffic counters)
python bench.py --mode batch   (64 uneven problems, N_b ~ U{2000..30000}, d_b ~ U{1..6},
    ARD RBF, 16 probes: MLL + gradient of every problem in one batched call)
python bench.py --mode rbf500k [--precision fp32|bf16x2|bf16x3] [--precond K]   (N = 500000, d = 2, RBF
    l = 0.05, 16 probes: one MLL + gradient in the chosen precision)
python bench.py --mode matvec   (K_y V entries/s: the 100k geometry at t = 1 and 33 in
    every precision, and N = 2k..50k at t = 1; the periodic family, one adjoint
    sweep per family, and kernel sums / products / Linear on the same points;
    HIP events around the whole call, median of 9 after ~100 ms of warm-up calls)
python bench.py --mode composite   (one MLL + gradient of Scale(RBF) + Scale(Periodic)
    on the 100k points, 32 probes)
python bench.py --mode variance   (predictive variance on the 100k points at 2000 test
    points, 32 probes)
python bench.py --mode ski   (structured kernel interpolation at N = 200000, D = 1 and 2:
    K_y V at t = 1 and 33, and a CG solve)
python bench.py --mode small   (end-to-end latency of the 1024-point RBF and the
    20000-point Matern-5/2 workloads: solve, MLL + gradient, predictive mean; the
    oracle's dense Cholesky route timed beside them)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X: 256 CU x 2.4 GHz x 256 FLOP/clk/CU (packed FP32 FMA)
# HBM bytes per launch of the step's dominant kernel (RBF, d = 4, t = 33,
# N = 100000), from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB copy's
# reading of the same counters (summaries in profiles/).  Valid only for the
# kernels named below.
HYB_TRAFFIC_BYTES = 2.664e8
GRAM_TRAFFIC_BYTES = 6.543e8
TRAFFIC_SOURCE = {
    "fp32": "profiles/sweep_gram_rbf_d4_t33_rbf100k.md (rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel, "
            "scaled by a 1 GiB copy's counters; taken from that profile, not measured in this run)",
    "fp32_direct": "profiles/sweep_hyb_rbf_d4_t33_rbf100k.md (same method; not measured in this run)",
}
BF16_MFMA_PEAK_TFLOPS = 2500.0   # MI355X dense bf16 matrix peak
# Dominant kernel of the step per precision: (name, bound, HBM bytes per launch).
STEP_KERNELS = {
    "fp32": ("sweep_gram_kernel<d=4, NT=2, TV=1> (RBF squared distances and the K-tile x V "
             "contraction on v_mfma_f32_16x16x4_f32, exp2 on the VALU)", "mfma", GRAM_TRAFFIC_BYTES),
    "fp32_direct": ("sweep_hyb_kernel<RBF, d=4, NT=2, TV=1> (FP32 entries from direct differences on "
                    "the VALU, contraction on v_mfma_f32_16x16x4_f32)", "alu", HYB_TRAFFIC_BYTES),
}
# Pipe utilisation of the dominant kernel from rocprofv3 SQ counters (taken
# from the named profile, not measured in this run): the matrix-core busy
# fraction and the VALU work beside it.
STEP_COUNTERS = {
    "fp32": {"mfma_busy": 0.742, "mfma_insts_per_64_entries": 2.25, "valu_insts_per_64_entries": 2.61,
             "valu_trans_per_64_entries": 1.00,
             "source": "profiles/sweep_gram_rbf_d4_t33_rbf100k.md (SQ_VALU_MFMA_BUSY_CYCLES / GRBM_GUI_ACTIVE, "
                       "SQ_INSTS_VALU*; not measured in this run)"},
    "fp32_direct": {"mfma_busy": 0.538, "valu_insts_per_64_entries": 11.3,
                    "source": "profiles/sweep_hyb_rbf_d4_t33_rbf100k.md (same counters; not measured in this run)"},
}
METRIC = "kernel entries/s and CG solve time at N=100k; MLL+grad time, BF16 vs FP32"
# SIMD cycles per wave64 instruction on gfx950 (paper_2605_17898_amd/issue_rates,
# profiles/issue_rates_gfx950.md): v_exp_f32 issues at half the FMA rate, and
# FP32 MFMA does not overlap the VALU, so a sweep's instruction counts priced at
# these rates and summed bound its cycles from below.
ISSUE_CYCLES = {"exp": 8.34, "valu": 4.21, "mfma_f32_16x16x4": 32.43}
# Instruction counts per 64 entries of the FP32 Gram sweep at t = 1 (rocprofv3
# SQ_INSTS_VALU*, profiles/sweep_gram_rbf_d4_t1_rbf100k.md; not measured in this run)
T1_COUNTERS = {"mfma_insts_per_64_entries": 0.25, "valu_insts_per_64_entries": 2.31,
               "valu_trans_per_64_entries": 1.00}


def issue_bound(counters: dict, launch_ms: float, entries: float) -> dict:
    """The sweep's cycles per 64 entries at the measured issue rates (exp2,
    other VALU, FP32 MFMA, summed) against the cycles one launch took at
    2.4 GHz over the 64-entry slots each of the 1024 SIMDs executes."""
    trans = counters["valu_trans_per_64_entries"]
    model = (trans * ISSUE_CYCLES["exp"] + (counters["valu_insts_per_64_entries"] - trans) * ISSUE_CYCLES["valu"]
             + counters["mfma_insts_per_64_entries"] * ISSUE_CYCLES["mfma_f32_16x16x4"])
    measured = launch_ms * 1e-3 * 2.4e9 / (entries / 64.0 / 1024.0)
    return {"model_cycles_per_64_entries": model, "measured_cycles_per_64_entries": measured,
            "frac": model / measured,
            "source": "profiles/issue_rates_gfx950.md (rates) and the counters' profile (counts)"}


def cpu_baseline(w, rows: int) -> dict:
    """Oracle FP64 K_y V on a bounded row sample of the step's t = 33 product."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import gp
    k = gp.Kern(w.family, w.lengthscale, w.outputscale, w.noise)
    V = np.concatenate([w.y[:, None], w.Z], axis=1).astype(np.float64)
    sel = np.random.default_rng(0).choice(w.n, size=rows, replace=False)
    t0 = time.perf_counter()
    gp.ky_matvec_rows(k, w.X, V, sel)
    dt = time.perf_counter() - t0
    blas = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
    return {"value": rows * w.n / dt, "unit": "entries/s", "cores": max(blas) if blas else 1,
            "kind": "oracle",
            "sample": f"FP64 K_y V for {rows} of {w.n} rows, t=33 (the step's product); "
                      f"{dt:.1f} s; numpy elementwise work is single-threaded, the BLAS product "
                      f"uses the reported threads"}


def batch_leg(args) -> int:
    """MLL + gradient of the 64-problem batch (one tuned persistent-launch call)."""
    import numpy as np
    import torch

    from paper_2605_17898_amd import inputs, mfgp
    probs = inputs.batch64(probes=16)
    X = torch.from_numpy(np.concatenate([w.X.reshape(-1) for w in probs])).cuda()
    y = torch.from_numpy(np.concatenate([w.y for w in probs])).cuda()
    Z = torch.from_numpy(np.concatenate([w.Z for w in probs])).cuda()
    plan = mfgp.BatchPlan([mfgp.Kernel(w.family, [float(v) for v in w.lengthscale], w.outputscale, w.noise)
                           for w in probs], [w.n for w in probs], [w.d for w in probs], 16, tune=True)
    def progress(it, rr):
        print(f"[bench] batch64: {it} iterations, worst recurrence residual {rr:.2e}",
              file=sys.stderr, flush=True)

    print("[bench] batch warm-up call (tunes the tile length)", file=sys.stderr, flush=True)
    plan.mll_and_grad(X, y, Z, progress=progress, precision=args.precision)
    torch.cuda.synchronize()
    mfgp.timing_enable(True)
    t0 = time.perf_counter()
    r = plan.mll_and_grad(X, y, Z, progress=progress, precision=args.precision)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ph = mfgp.timing_phases()
    mfgp.timing_enable(False)
    entries = sum(float(w.n) ** 2 for w in probs)
    print(json.dumps({"mode": "batch", "workload": "batch64", "precision": args.precision, "problems": len(probs),
                      "rows": int(sum(w.n for w in probs)), "entries_per_product": entries,
                      "mll_grad_s": el, "cg_s": ph["cg_ms"] * 1e-3, "slq_s": ph["slq_ms"] * 1e-3,
                      "adjoint_s": ph["adjoint_ms"] * 1e-3, "status": r["status"], "plan": plan.info(),
                      "cg_iters_max": max(max(i["iters"] for i in inf) for inf in r["info"]),
                      "rel_resid_true_max": max(max(i["rel_resid_true"] for i in inf) for inf in r["info"])}))
    return 0


def rbf500k_leg(args) -> int:
    """One MLL + gradient on N = 500000 (16 probes), FP32 or BF16-x2, with solver progress."""
    import torch

    from paper_2605_17898_amd import inputs, mfgp
    w = inputs.rbf500k()
    kern = mfgp.Kernel(w.family, w.lengthscale, w.outputscale, w.noise)
    X = torch.from_numpy(w.X).cuda()
    y = torch.from_numpy(w.y).cuda()
    Z = torch.from_numpy(w.Z).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def progress(it, rr):
        print(f"[bench] rbf500k {args.precision}: {it} iterations, worst recurrence residual {rr:.2e}, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    mfgp.timing_enable(True)
    factor_s = None
    if args.precond > 0:
        # rank-k pivoted-Cholesky preconditioner; probes z ~ N(0, P) from
        # standard normal draws (the preconditioned estimator's probes)
        L, _ = mfgp.pivoted_cholesky(kern, X, args.precond)
        E = torch.from_numpy(inputs.gaussian_rhs(411, args.precond, Z.shape[1])).cuda()
        G = torch.from_numpy(inputs.gaussian_rhs(412, w.n, Z.shape[1])).cuda()
        Zp = mfgp.precond_probes(L, w.noise, E, G)
        torch.cuda.synchronize()
        factor_s = time.perf_counter() - t0
        r = mfgp.precond_mll_and_grad(kern, X, y, Zp, L, tol=1e-6, precision=args.precision, progress=progress)
    else:
        r = mfgp.mll_and_grad(kern, X, y, Z=Z, tol=1e-6, precision=args.precision, progress=progress)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ph = mfgp.timing_phases()
    allk = mfgp.timing_read(-1)
    mfgp.timing_enable(False)
    print(json.dumps({"mode": "rbf500k", "precision": args.precision, "n": w.n, "probes": 16,
                      "precond_rank": args.precond, "factor_s": factor_s,
                      "mll_grad_s": el, "cg_s": ph["cg_ms"] * 1e-3, "slq_s": ph["slq_ms"] * 1e-3,
                      "adjoint_s": ph["adjoint_ms"] * 1e-3, "status": r["status"],
                      "cg_iters_max": max(i["iters"] for i in r["info"]),
                      "rel_resid_true_max": max(i["rel_resid_true"] for i in r["info"]),
                      "cg_refinements_max": max(i["refinements"] for i in r["info"]),
                      "stalls_max": max(i["stalls"] for i in r["info"]),
                      "precision_final": sorted({i["precision"] for i in r["info"]}),
                      "entries_per_s": allk["entries"] / el, "mll": r["mll"], "logdet": r["logdet"],
                      "grad": r["grad"]}))
    return 0


def ski_leg(args) -> int:
    """Structured kernel interpolation at N = 200000 (D = 1, and D = 2 on a
    280 x 280 grid): the whole K_y V call at t = 1 and 33, and a CG solve of y
    to 1e-6."""
    import torch

    from paper_2605_17898_amd import inputs, mfgp
    rows = []
    for d, grids in ((1, ([10000], [100000])), (2, ([280, 280],))):
        w = inputs.ski200k(d=d)
        kern = mfgp.Kernel(w.family, w.lengthscale, w.outputscale, w.noise)
        X = torch.from_numpy(w.X).cuda()
        y = torch.from_numpy(w.y).cuda()
        for m in grids:
            g = mfgp.ski_grid(m)
            for t in (1, 33):
                V = torch.randn(w.n, t, device="cuda") if t > 1 else y.clone()
                out = torch.empty_like(V)
                ms = _median_call_ms(lambda: mfgp.ski_matvec(kern, X, V, g, out=out))
                rows.append({"d": d, "m": m, "n": w.n, "t": t, "matvec_ms": ms})
                print(f"[bench] ski matvec d={d} m={m} t={t}: {ms:.3f} ms", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info, st = mfgp.ski_cg_solve(kern, X, y, g, tol=1e-6)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            rows.append({"d": d, "m": m, "n": w.n, "cg_solve_s": el, "iters": info[0]["iters"],
                         "rel_resid_true": info[0]["rel_resid_true"], "status": st})
            print(f"[bench] ski cg d={d} m={m}: {el:.3f} s, {info[0]['iters']} iterations", file=sys.stderr,
                  flush=True)
    print(json.dumps({"mode": "ski", "workload": "ski200k (uniform [0,1]^d, RBF l=0.05, sigma^2=0.01)",
                      "rows": rows}))
    return 0


def variance_leg(args) -> int:
    """Predictive variance on the rbf100k points at its 2000 test points with
    32 seeded Rademacher probes (one CG solve of 32 columns between two
    rectangular sweeps), FP32 and with the Gram-form solve."""
    import torch

    from paper_2605_17898_amd import inputs, mfgp
    w = inputs.rbf100k()
    kern = mfgp.Kernel(w.family, w.lengthscale, w.outputscale, w.noise)
    X = torch.from_numpy(w.X).cuda()
    Xs = torch.from_numpy(w.Xs).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    var, info, st = mfgp.predict_variance(kern, X, Xs, num_probes=32, seed=7, tol=1e-6)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    v = var.double()
    # ground truth on the first 64 test points: identity probes make the
    # estimator exact (up to the CG tolerance)
    Xe = Xs[:64].contiguous()
    eye = torch.eye(64, dtype=torch.float32, device="cuda")
    t1 = time.perf_counter()
    ve, info_e, st_e = mfgp.predict_variance(kern, X, Xe, Z=eye, tol=1e-6)
    torch.cuda.synchronize()
    el_e = time.perf_counter() - t1
    # the 32-probe estimate restricted to the same 64 points (same estimator, 64 test points)
    vs, _, _ = mfgp.predict_variance(kern, X, Xe, num_probes=32, seed=7, tol=1e-6)
    err = (vs.double() - ve.double()).abs()
    print(json.dumps({"mode": "variance", "workload": "rbf100k, 2000 test points, 32 probes", "seconds": el,
                      "status": st, "cg_iters_max": max(i["iters"] for i in info),
                      "rel_resid_true_max": max(i["rel_resid_true"] for i in info),
                      "var_min": float(v.min()), "var_mean": float(v.mean()), "var_max": float(v.max()),
                      "exact_64": {"seconds": el_e, "status": st_e, "cg_iters_max": max(i["iters"] for i in info_e),
                                   "var_min": float(ve.min()), "var_max": float(ve.max()),
                                   "probe32_on_same_64_max_abs_err": float(err.max()),
                                   "probe32_on_same_64_mean_abs_err": float(err.mean())}}))
    return 0


def composite_leg(args) -> int:
    """One MLL + gradient of Scale(RBF) + Scale(Periodic) on the rbf100k points
    ([y, 32 probes], tol 1e-6): the paper's composition example at N = 1e5."""
    import torch

    from paper_2605_17898_amd import inputs, mfgp
    w = inputs.rbf100k()
    kern = (mfgp.Kernel("rbf", w.lengthscale, w.outputscale, w.noise)
            + mfgp.Kernel("periodic", 1.0, 0.5 * w.outputscale, period=0.5))
    X = torch.from_numpy(w.X).cuda()
    y = torch.from_numpy(w.y).cuda()
    Z = torch.from_numpy(w.Z).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def progress(it, rr):
        print(f"[bench] composite: {it} iterations, worst recurrence residual {rr:.2e}, "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    mfgp.timing_enable(True)
    r = mfgp.mll_and_grad(kern, X, y, Z=Z, tol=1e-6, progress=progress)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ph = mfgp.timing_phases()
    f32 = mfgp.timing_read(mfgp.SWEEP_F32)
    adj = mfgp.timing_read(mfgp.SWEEP_ADJOINT)
    mfgp.timing_enable(False)
    print(json.dumps({"mode": "composite", "kernel": "rbf(l=0.3) + periodic(l=1, p=0.5, s2/2)", "n": w.n,
                      "probes": int(Z.shape[1]), "mll_grad_s": el, "cg_s": ph["cg_ms"] * 1e-3,
                      "slq_s": ph["slq_ms"] * 1e-3, "adjoint_s": ph["adjoint_ms"] * 1e-3, "status": r["status"],
                      "cg_iters_max": max(i["iters"] for i in r["info"]),
                      "rel_resid_true_max": max(i["rel_resid_true"] for i in r["info"]),
                      "sweep_launches": f32["launches"], "sweep_ms_avg": f32["ms"] / max(f32["launches"], 1),
                      "adjoint_sweep_ms": adj["ms"], "mll": r["mll"], "logdet": r["logdet"], "grad": r["grad"]}))
    return 0


def _warm(fn, min_ms: float = 100.0, max_calls: int = 400) -> None:
    """Run fn() back to back for about min_ms: the GPU raises its clocks under
    sustained load, and a short burst after idle runs up to 15% slower (the
    t = 1 product: 1.80 ms per call after 2 s idle, 1.55 ms sustained)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max_calls):
        fn()
        torch.cuda.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= min_ms:
            break


def _median_call_ms(fn, reps: int = 9, warm: bool = True) -> float:
    """Median wall time of fn() bracketed by events on torch's current stream,
    after about 100 ms of warm-up calls (one call if warm is False)."""
    import torch
    if warm:
        _warm(fn)
    else:
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def matvec_leg(args) -> int:
    """Entries/s of the whole K_y V call (prescale, packing, sweep, reduction)."""
    import numpy as np
    import torch

    from paper_2605_17898_amd import inputs, mfgp
    rows = []
    full = inputs.rbf100k()
    kern = mfgp.Kernel(full.family, full.lengthscale, full.outputscale, full.noise)
    Xf = torch.from_numpy(full.X).cuda()
    Vall = torch.from_numpy(np.concatenate([full.y[:, None], full.Z], axis=1)).cuda()
    cases = [(full.n, t, prec) for t in (1, 33)
             for prec in ("fp32", "fp32_direct", "fp32_valu", "bf16x1", "bf16x2", "bf16x3")]
    cases += [(n, 1, prec) for n in (2000, 5000, 10000, 20000, 50000) for prec in ("fp32_gram", "fp32_direct")]
    for n, t, prec in cases:
        X = Xf[:n].contiguous()
        V = Vall[:n, :t].contiguous()
        out = torch.empty_like(V)
        ms = _median_call_ms(lambda: mfgp.kernel_matvec(kern, X, V, precision=prec, out=out))
        rows.append({"n": n, "t": t, "precision": prec, "ms": ms, "entries_per_s": n * n / (ms * 1e-3),
                     "rhs_products_per_s": n * n * t / (ms * 1e-3),
                     "tflops": n * n * (3 * 4 + 1 + 2 * t) / (ms * 1e-3) / 1e12})
        print(f"[bench] matvec n={n} t={t} {prec}: {ms:.3f} ms", file=sys.stderr, flush=True)
    # the periodic family on the same points: RBF sweeps over its 8 circle features
    pk = mfgp.Kernel("periodic", 1.0, full.outputscale, full.noise, period=0.5)
    prow = []
    for t, prec in ((1, "fp32"), (33, "fp32"), (33, "fp32_direct"), (33, "bf16x2")):
        V = Vall[:, :t].contiguous()
        out = torch.empty_like(V)
        ms = _median_call_ms(lambda: mfgp.kernel_matvec(pk, Xf, V, precision=prec, out=out))
        n = full.n
        prow.append({"n": n, "t": t, "precision": prec, "ms": ms, "entries_per_s": n * n / (ms * 1e-3),
                     "tflops": n * n * (3 * 8 + 1 + 2 * t) / (ms * 1e-3) / 1e12})
        print(f"[bench] periodic matvec n={n} t={t} {prec}: {ms:.3f} ms", file=sys.stderr, flush=True)
    # one adjoint sweep (t = 33: [alpha, 32 probes]) per family: the periodic
    # sweep adds the period term to the paired lengthscale terms
    A = Vall.contiguous()
    arow = []
    for name, k in (("rbf", kern), ("periodic", pk)):
        ms = _median_call_ms(lambda: mfgp.kernel_adjoint(k, Xf, A, A, [0.5] + [-0.5 / 32] * 32))
        arow.append({"family": name, "n": full.n, "t": 33, "ms": ms})
        print(f"[bench] adjoint {name} n={full.n} t=33: {ms:.3f} ms", file=sys.stderr, flush=True)
    # compositions (the paper's Scale(RBF) + Scale(Periodic), a product of two
    # RBF factors, Linear) on the same points
    comps = (("rbf(l=0.3) + periodic(l=1, p=0.5)", kern + pk, (1, 33)),
             ("rbf(l=0.3) * rbf(l=0.8) (8 features)",
              mfgp.Kernel("rbf", 0.3, full.outputscale, full.noise) * mfgp.Kernel("rbf", 0.8), (1, 33)),
             ("matern52(l=0.3) * rbf(l=0.8) (general product, 8 features)",
              mfgp.Kernel("matern52", 0.3, full.outputscale, full.noise) * mfgp.Kernel("rbf", 0.8), (1, 33)),
             ("linear", mfgp.Kernel("linear", 1.0, 1.0, full.noise), (1, 33)))
    crow = []
    for name, k, ts in comps:
        for t in ts:
            V = Vall[:, :t].contiguous()
            out = torch.empty_like(V)
            ms = _median_call_ms(lambda: mfgp.kernel_matvec(k, Xf, V, out=out))
            crow.append({"kernel": name, "n": full.n, "t": t, "ms": ms})
            print(f"[bench] {name} matvec n={full.n} t={t}: {ms:.3f} ms", file=sys.stderr, flush=True)
    print(json.dumps({"mode": "matvec", "workload": "rbf100k geometry (d=4, RBF l=0.3)", "rows": rows,
                      "periodic": {"kernel": "periodic d=4 l=1.0 p=0.5 (8 features)", "rows": prow},
                      "adjoint": arow, "compositions": crow}))
    return 0


def small_leg(args) -> int:
    """End-to-end latency at N = 1024 (RBF) and N = 20000 (Matern-5/2), oracle beside."""
    import numpy as np
    import torch

    from oracle import gp
    from paper_2605_17898_amd import inputs, mfgp
    out = []
    for name, w in (("exact1k", inputs.exact1k(probes=16)), ("matern20k", inputs.matern20k(probes=16))):
        kern = mfgp.Kernel(w.family, w.lengthscale, w.outputscale, w.noise)
        X = torch.from_numpy(w.X).cuda()
        y = torch.from_numpy(w.y).cuda()
        Z = torch.from_numpy(w.Z).cuda()
        Xs = torch.from_numpy(w.Xs).cuda() if w.Xs is not None else X
        box = {}

        def solve():
            box["x"], box["info"], _, _ = mfgp.cg_solve(kern, X, y, tol=1e-6)

        def mll():
            box["m"] = mfgp.mll_and_grad(kern, X, y, Z=Z, tol=1e-6)

        def mean():
            mfgp.predict_mean(kern, X, Xs, box["x"].float())

        rec = {"workload": name, "n": w.n, "d": w.d, "family": w.family, "probes": int(Z.shape[1]),
               "solve_ms": _median_call_ms(solve), "solve_iters": box["info"][0]["iters"],
               "solve_rel_resid_true": box["info"][0]["rel_resid_true"],
               "mll_grad_ms": _median_call_ms(mll), "predict_mean_ms": _median_call_ms(mean),
               "test_points": int(Xs.shape[0])}
        print(f"[bench] {name} GPU done; oracle", file=sys.stderr, flush=True)
        k = gp.Kern(w.family, w.lengthscale, w.outputscale, w.noise)
        t0 = time.perf_counter()
        ch = gp.cholesky(k, w.X)
        alpha = gp.solve(k, w.X, w.y, chol=ch)
        ld = gp.logdet(k, w.X, chol=ch)
        rec["oracle_solve_logdet_s"] = time.perf_counter() - t0
        rec["oracle_route"] = "FP64 dense K_y, Cholesky, two triangular solves, log-det"
        rec["alpha_rel_err_vs_oracle"] = float(np.linalg.norm(box["x"].cpu().numpy().ravel() - alpha) /
                                               np.linalg.norm(alpha))
        rec["logdet_oracle"] = float(ld)
        rec["logdet_slq"] = box["m"]["logdet"]
        out.append(rec)
        print(f"[bench] {name} oracle done", file=sys.stderr, flush=True)
    print(json.dumps({"mode": "small", "rows": out}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32",
                    choices=["fp32", "fp32_direct", "fp32_valu", "bf16x1", "bf16x2", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=10240)
    ap.add_argument("--mode", default="step",
                    choices=["step", "kernel", "batch", "rbf500k", "matvec", "small", "composite", "ski",
                             "variance"])
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison steps (direct-difference FP32, BF16-x2, BF16-x3, preconditioned)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cols", type=int, default=33,
                    help="kernel mode: right-hand sides of the product ([y, probes][:cols], 1..33)")
    ap.add_argument("--compare-reps", type=int, default=5,
                    help="runs of each comparison step (the median is reported)")
    ap.add_argument("--precond", type=int, default=0,
                    help="rbf500k mode: rank of a pivoted-Cholesky preconditioner (0: plain CG)")
    ap.add_argument("--pc-rank", type=int, default=1024,
                    help="rank of the preconditioned comparison step (0 skips it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of the path is a design note, not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2605_17898_amd import inputs, mfgp

    torch.cuda.set_device(0)
    if args.mode == "batch":
        return batch_leg(args)
    if args.mode == "rbf500k":
        return rbf500k_leg(args)
    if args.mode == "ski":
        return ski_leg(args)
    if args.mode == "variance":
        return variance_leg(args)
    if args.mode == "composite":
        return composite_leg(args)
    if args.mode == "matvec":
        return matvec_leg(args)
    if args.mode == "small":
        return small_leg(args)
    w = inputs.rbf100k()
    kern = mfgp.Kernel(w.family, w.lengthscale, w.outputscale, w.noise)
    X = torch.from_numpy(w.X).cuda()
    y = torch.from_numpy(w.y).cuda()
    Z = torch.from_numpy(w.Z).cuda()
    Xs = torch.from_numpy(w.Xs).cuda()
    torch.cuda.synchronize()

    if args.mode == "kernel":
        V = torch.cat([y[:, None], Z], dim=1)[:, :args.cols].contiguous()
        for i in range(args.reps):
            mfgp.kernel_matvec(kern, X, V, precision=args.precision)
            torch.cuda.synchronize()
            print(f"[bench] kernel launch {i + 1}/{args.reps}", file=sys.stderr, flush=True)
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "kernel", "reps": args.reps, "copy_bytes": src.numel() * 4}))
        return 0

    def step():
        r = mfgp.mll_and_grad(kern, X, y, Z=Z, tol=1e-6, precision=args.precision, want_alpha=True)
        mu = mfgp.predict_mean(kern, X, Xs, r["alpha"].float())
        return r, mu

    for i in range(args.warmup):
        print(f"[bench] warmup step {i + 1}/{args.warmup}", file=sys.stderr, flush=True)
        step()
    torch.cuda.synchronize()

    mfgp.timing_enable(True)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        results.append(step())
        torch.cuda.synchronize()
        print(f"[bench] timed step {i + 1}/{args.steps} done at {time.perf_counter() - t0:.2f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    allk = mfgp.timing_read(-1)
    f32 = mfgp.timing_read(mfgp.SWEEP_F32)
    f64 = mfgp.timing_read(mfgp.SWEEP_F64)
    adj = mfgp.timing_read(mfgp.SWEEP_ADJOINT)
    mfma = mfgp.timing_read(mfgp.SWEEP_MFMA)
    ph = mfgp.timing_phases()
    mfgp.timing_enable(False)

    r = results[-1][0]
    info = r["info"]
    dom = f32 if args.precision.startswith("fp32") else mfma
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12 if dom["ms"] > 0 else 0.0
    line = {
        "metric": METRIC,
        "value": allk["entries"] / elapsed,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": "rbf100k", "n": w.n, "d": w.d, "family": "rbf", "lengthscale": 0.3,
                   "noise": 0.01, "probes": 32, "t": 33, "tol": 1e-6, "test_points": w.Xs.shape[0],
                   "precision": args.precision},
        "cg_solve_s": ph["cg_ms"] * 1e-3 / args.steps,
        "mll_grad_s": (ph["cg_ms"] + ph["slq_ms"] + ph["adjoint_ms"]) * 1e-3 / args.steps,
        "slq_s": ph["slq_ms"] * 1e-3 / args.steps,
        "adjoint_s": ph["adjoint_ms"] * 1e-3 / args.steps,
        "cg_iters_max": max(i["iters"] for i in info),
        "cg_refinements_max": max(i["refinements"] for i in info),
        "cg_replacements_max": max(i["replacements"] for i in info),
        "cg_drift_skips_max": max(i["drift_skips"] for i in info),
        "precision_final": sorted({i["precision"] for i in info}),
        "rel_resid_true_max": max(i["rel_resid_true"] for i in info),
        "mll": r["mll"],
        "logdet": r["logdet"],
        "matvec_sweeps_per_step": f32["launches"] / args.steps,
        "matvec_sweep_ms_avg": f32["ms"] / max(f32["launches"], 1),
        "matvec_entries_per_s": f32["entries"] / (f32["ms"] * 1e-3) if f32["ms"] > 0 else 0.0,
        "sweep_ms": {"fp32": f32["ms"], "fp64acc": f64["ms"], "adjoint": adj["ms"], "mfma": mfma["ms"]},
        "roofline": {
            "bound": STEP_KERNELS.get(args.precision, ("", "mfma", None))[1],
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": STEP_KERNELS.get(args.precision, ("", "", None))[2],
            "traffic_unit": "bytes per launch",
            "traffic_source": TRAFFIC_SOURCE.get(args.precision),
            "peak_note": "MI355X FP32 peak (157.3 TFLOP/s, vector with packed FMA; the FP32 matrix cores have "
                         "the same rate); the Gram form runs 78 of the 79 FLOP per entry on FP32 MFMA",
            "kernel": STEP_KERNELS.get(args.precision, ("bf16 mfma sweep", "", None))[0],
            "flop_per_entry": 3 * 4 + 1 + 2 * 33,
            "launch_avg_ms": dom["ms"] / max(dom["launches"], 1),
            "counters": STEP_COUNTERS.get(args.precision),
        },
    }
    if args.precision == "fp32":
        line["roofline"]["issue_bound"] = issue_bound(STEP_COUNTERS["fp32"], line["roofline"]["launch_avg_ms"],
                                                      float(w.n) * float(w.n))
    if args.precision == "fp32":
        # The paper's Table 3 product on this geometry: K_y v with one
        # right-hand side (RBF, d = 4, N = 1e5), median of 9 calls after about
        # 100 ms of warm-up calls (sustained clocks, as inside a solve); the
        # sweep kernel's own time from events on its stream.
        v1 = y.reshape(-1, 1).contiguous()
        o1 = torch.empty_like(v1)
        _warm(lambda: mfgp.kernel_matvec(kern, X, v1, out=o1))
        mfgp.timing_enable(True)
        ms1 = _median_call_ms(lambda: mfgp.kernel_matvec(kern, X, v1, out=o1), warm=False)
        k1 = mfgp.timing_read(mfgp.SWEEP_F32)
        mfgp.timing_enable(False)
        sw1 = k1["ms"] / max(k1["launches"], 1)
        fl1 = 3 * w.d + 1 + 2
        ach1 = float(w.n) * float(w.n) * fl1 / (sw1 * 1e-3) / 1e12
        line["table3_t1"] = {
            "workload": "rbf100k geometry at t = 1 (Table 3's product: RBF, D = 4, one right-hand side)",
            "call_ms_median": ms1,
            "entries_per_s": float(w.n) * float(w.n) / (ms1 * 1e-3),
            "roofline": {"bound": "alu", "kernel": "sweep_gram_kernel<d=4, NT=0, TV=1> (squared distances on "
                                                   "v_mfma_f32_16x16x4_f32; exp2 and the FMA on the VALU)",
                         "flop_per_entry": fl1, "achieved": ach1, "peak": FP32_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach1 / FP32_VECTOR_PEAK_TFLOPS, "launch_avg_ms": sw1,
                         "issue_bound": issue_bound(T1_COUNTERS, sw1, float(w.n) * float(w.n))},
        }
        print(f"[bench] t=1 product: {ms1:.3f} ms per call, sweep {sw1:.3f} ms", file=sys.stderr, flush=True)
    if args.precision == "fp32" and not args.no_compare:
        # The same step with the K-tile x V contraction on the bf16 matrix cores
        # (FP32 entries, FP64-accumulated residual replacement and refinement to
        # the same 1e-6): the hi/lo split (x2) and the exact three-way split (x3);
        # and the FP32 form with direct differences.  Median of --compare-reps
        # runs of each (by step time).
        for form in ("fp32_direct", "bf16x2", "bf16x3"):
            reps = []
            for rep in range(args.compare_reps):
                print(f"[bench] {form} comparison step {rep + 1}/{args.compare_reps}", file=sys.stderr, flush=True)
                torch.cuda.synchronize()
                mfgp.timing_enable(True)
                t1 = time.perf_counter()
                rb = mfgp.mll_and_grad(kern, X, y, Z=Z, tol=1e-6, precision=form, want_alpha=True)
                mfgp.predict_mean(kern, X, Xs, rb["alpha"].float())
                torch.cuda.synchronize()
                eb = time.perf_counter() - t1
                ab = mfgp.timing_read(-1)
                mb = mfgp.timing_read(mfgp.SWEEP_F32 if form.startswith("fp32") else mfgp.SWEEP_MFMA)
                phb = mfgp.timing_phases()
                mfgp.timing_enable(False)
                sweep_ms = mb["ms"] / max(mb["launches"], 1)
                leg = {
                    "ms_per_step": eb * 1e3,
                    "entries_per_s": ab["entries"] / eb,
                    "cg_solve_s": phb["cg_ms"] * 1e-3,
                    "mll_grad_s": (phb["cg_ms"] + phb["slq_ms"] + phb["adjoint_ms"]) * 1e-3,
                    "cg_iters_max": max(i["iters"] for i in rb["info"]),
                    "cg_refinements_max": max(i["refinements"] for i in rb["info"]),
                    "rel_resid_true_max": max(i["rel_resid_true"] for i in rb["info"]),
                    "precision_final": sorted({i["precision"] for i in rb["info"]}),
                    "sweep_ms_avg": sweep_ms,
                    "sweep_entries_per_s": mb["entries"] / (mb["ms"] * 1e-3) if mb["ms"] > 0 else 0.0,
                    "mll": rb["mll"],
                    "logdet": rb["logdet"],
                }
                if form.startswith("bf16") and sweep_ms > 0:
                    # entries on the VALU (3d + 1 FLOP, + 2 for the FP32 y column),
                    # the 32 probe columns contracted on the bf16 matrix cores
                    # (2 FLOP per entry and column), reported against each unit's peak
                    ent = float(w.n) * float(w.n)
                    gen = ent * (3 * w.d + 1 + 2) / (sweep_ms * 1e-3) / 1e12
                    con = ent * 2 * 32 / (sweep_ms * 1e-3) / 1e12
                    leg["roofline"] = {
                        "kernel": f"sweep_gmfma_kernel ({form}: Gram distances on v_mfma_f32_32x32x2_f32, "
                                  "exp2 and the bf16 split on the VALU, K-tile x V on v_mfma_f32_32x32x16_bf16)",
                        "valu_generation": {"flop_per_entry": 3 * w.d + 3, "achieved": gen,
                                            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                            "frac": gen / FP32_VECTOR_PEAK_TFLOPS},
                        "contraction": {"flop_per_entry": 64, "achieved": con, "peak": BF16_MFMA_PEAK_TFLOPS,
                                        "unit": "TFLOP/s", "frac": con / BF16_MFMA_PEAK_TFLOPS},
                        "launch_avg_ms": sweep_ms,
                    }
                reps.append(leg)
            reps.sort(key=lambda d: d["ms_per_step"])
            med = dict(reps[len(reps) // 2])
            med["reps"] = len(reps)
            med["ms_per_step_all"] = [d["ms_per_step"] for d in reps]
            line[form] = med
    if args.precision == "fp32" and not args.no_compare and args.pc_rank > 0:
        # The same MLL + gradient with the rank-k pivoted-Cholesky preconditioner
        # (factor build, probes z ~ N(0, P), preconditioned CG, SLQ, adjoint):
        # what the unpreconditioned CG of the paper lacks.
        print(f"[bench] preconditioned step, rank {args.pc_rank}", file=sys.stderr, flush=True)
        k = args.pc_rank
        E = torch.from_numpy(inputs.gaussian_rhs(401, k, Z.shape[1])).cuda()
        G = torch.from_numpy(inputs.gaussian_rhs(402, w.n, Z.shape[1])).cuda()
        torch.cuda.synchronize()
        mfgp.timing_enable(True)
        t1 = time.perf_counter()
        L, _ = mfgp.pivoted_cholesky(kern, X, k)
        Zp = mfgp.precond_probes(L, w.noise, E, G)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t1
        rp = mfgp.precond_mll_and_grad(kern, X, y, Zp, L, tol=1e-6, want_alpha=True)
        mfgp.predict_mean(kern, X, Xs, rp["alpha"].float())
        torch.cuda.synchronize()
        ep = time.perf_counter() - t1
        php = mfgp.timing_phases()
        mfgp.timing_enable(False)
        line[f"pcg_rank{k}"] = {
            "ms_per_step": ep * 1e3,
            "factor_s": tb,
            "cg_solve_s": php["cg_ms"] * 1e-3,
            "mll_grad_s": (php["cg_ms"] + php["slq_ms"] + php["adjoint_ms"]) * 1e-3,
            "cg_iters_max": max(i["iters"] for i in rp["info"]),
            "cg_refinements_max": max(i["refinements"] for i in rp["info"]),
            "rel_resid_true_max": max(i["rel_resid_true"] for i in rp["info"]),
            "mll": rp["mll"],
            "logdet": rp["logdet"],
            "probes": "z ~ N(0, P) (Gaussian), not the Rademacher probes of the FP32 step",
        }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on a bounded sample)", file=sys.stderr, flush=True)
        cb = cpu_baseline(w, args.cpu_rows)
        # the oracle's matrix-free CG is not run at this size: its solve time is
        # extrapolated as the GPU's product count times one oracle product
        oracle_matvec_s = float(w.n) * float(w.n) / cb["value"]
        cb["extrapolated"] = {"oracle_matvec_s": oracle_matvec_s,
                              "cg_solve_s": oracle_matvec_s * line["cg_iters_max"],
                              "note": "extrapolated: GPU CG iteration count x one oracle FP64 K_y V "
                                      "(t = 33) at the sampled rate; not measured"}
        line["cpu_baseline"] = cb
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
