"""Host-side checks that need no GPU: batch-plan argument validation (done
before any device call) and the benchmark's single-GPU contract."""

import ctypes as C
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_PATH = os.path.join(ROOT, "paper_2605_17898_amd", "libmfgp.so")


@pytest.fixture(scope="module")
def m():
    if not os.path.exists(LIB_PATH):
        pytest.skip("libmfgp.so not built")
    from paper_2605_17898_amd import mfgp
    return mfgp


def _create(m, ns, ds, kerns, probes=7, row_off=None, max_iter=0):
    nprob = len(ns)
    ro = row_off if row_off is not None else [sum(ns[:b]) for b in range(nprob)]
    xo = [sum(n * d for n, d in zip(ns[:b], ds[:b])) for b in range(nprob)]
    arrs = ((C.c_int64 * nprob)(*ns), (C.c_int64 * nprob)(*ro), (C.c_int64 * nprob)(*xo),
            (m.KernelT * nprob)(*[k.struct(d) for k, d in zip(kerns, ds)]))
    bt = m.BatchT(nprob, 0, *arrs)
    plan = C.c_void_p()
    st = m.LIB.mfgp_batch_plan_create(C.byref(bt), probes, max_iter, 0, 0, C.byref(plan))
    if plan.value:
        m.LIB.mfgp_batch_plan_destroy(plan)
    return st


def test_batch_plan_validation(m):
    k = m.Kernel("rbf", 0.3, 1.0, 0.01)
    assert _create(m, [100, 50], [2, 3], [k, k]) == m.OK
    assert _create(m, [100, 50], [2, 3], [k, k], probes=8) == m.UNSUPPORTED        # t = 9
    assert _create(m, [100, 50], [2, 3], [k, k], probes=0) == m.ERR_ARG
    assert _create(m, [100, 50], [2, 3], [k, k], max_iter=-1) == m.ERR_ARG
    assert _create(m, [100, 0], [2, 3], [k, k]) == m.ERR_ARG
    assert _create(m, [100, 50], [2, 9], [k, k]) == m.ERR_ARG
    assert _create(m, [100, 50], [2, 3], [k, m.Kernel("matern52", 0.3)]) == m.ERR_ARG
    assert _create(m, [100, 50], [2, 3], [k, m.Kernel("rbf", -0.3)]) == m.ERR_ARG
    assert _create(m, [100, 50], [2, 3], [k, m.Kernel("rbf", 0.3, 1.0, 0.0)]) == m.ERR_ARG
    assert _create(m, [100, 50], [2, 3], [k, k], row_off=[0, 120]) == m.ERR_ARG     # gap
    assert _create(m, [100, 50], [2, 3], [k, k], row_off=[50, 0]) == m.ERR_ARG      # reordered
    st = m.LIB.mfgp_batch_plan_create(None, 7, 0, 0, 0, C.byref(C.c_void_p()))
    assert st == m.ERR_ARG
    kp = m.Kernel("periodic", 0.3, 1.0, 0.01, period=0.5)
    assert _create(m, [100, 50], [2, 3], [kp, kp]) == m.UNSUPPORTED                 # not batched
    kl = m.Kernel("linear", 1.0, 1.0, 0.01)
    assert _create(m, [100, 50], [2, 3], [kl, kl]) == m.UNSUPPORTED
    ks = k + k
    assert _create(m, [100, 50], [2, 3], [ks, ks]) == m.UNSUPPORTED
    kx = k * k
    assert _create(m, [100, 50], [2, 3], [kx, kx]) == m.UNSUPPORTED
    # per-problem fragment indices are 32-bit: at most 2^24 rows per problem
    # (host validation only; nothing is allocated)
    assert _create(m, [2 ** 24, 50], [1, 3], [k, k]) == m.OK
    assert _create(m, [2 ** 24 + 1, 50], [1, 3], [k, k]) == m.UNSUPPORTED


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_issue_bound_prices_the_counted_instructions():
    # one exp2, two other VALU and two FP32 MFMA per 64 entries, for a launch
    # that took exactly the cycles they cost: the bound equals the measurement
    sys.path.insert(0, ROOT)
    import bench
    rates = bench.ISSUE_CYCLES
    c = {"valu_trans_per_64_entries": 1.0, "valu_insts_per_64_entries": 3.0, "mfma_insts_per_64_entries": 2.0}
    model = rates["exp"] + 2.0 * rates["valu"] + 2.0 * rates["mfma_f32_16x16x4"]
    entries = 64.0 * 1024.0 * 1000.0           # 1000 slots of 64 entries per SIMD
    launch_ms = model * 1000.0 / 2.4e9 * 1e3    # those slots at the model's cycles and 2.4 GHz
    ib = bench.issue_bound(c, launch_ms, entries)
    assert abs(ib["model_cycles_per_64_entries"] - model) < 1e-9
    assert abs(ib["measured_cycles_per_64_entries"] - model) < 1e-6
    assert abs(ib["frac"] - 1.0) < 1e-9
    # twice as long a launch halves the fraction
    assert abs(bench.issue_bound(c, 2 * launch_ms, entries)["frac"] - 0.5) < 1e-9
