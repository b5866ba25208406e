"""Gram form of the FP32 RBF sweep (squared distances on FP32 MFMA) against
the FP64 oracle, at the FP32 matvec bar: per-column relative error <= 1e-5.

The form computes r2 = |g_i|^2 + |g_j|^2 - 2 g_i.g_j from mean-centred
prescaled points, factored as 2^(-|g_i|^2) 2^(2 g_i.g_j) 2^(-|g_j|^2), while
max |g|^2 <= 62, and direct differences above; the launch picks the branch
from the maximum it computes.  Both branches are exercised here.
"""

import numpy as np
import pytest

from oracle import gp
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, col_rel_err, dev, host, mkern, okern

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


@pytest.mark.parametrize("t", [1, 16, 17, 33, 48, 49, 64, 65])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8])
def test_gram_matches_oracle(mf, d, t):
    # n = 3001: a ragged last 16-j block and a ragged last row block
    banner(f"matvec fp32_gram rbf d={d} n=3001 t={t}")
    w = inputs.random_problem(600 + d, 3001, d, "rbf", ard=True)
    V = inputs.gaussian_rhs(610 + t, 3001, t)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="fp32_gram"))
    ref = gp.ky_matrix(okern(w), w.X) @ V.astype(np.float64)
    assert col_rel_err(out, ref).max() <= TOL


@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 255, 257])
def test_gram_small_and_ragged(mf, n):
    banner(f"matvec fp32_gram rbf d=3 n={n} t=17")
    w = inputs.random_problem(620, n, 3, "rbf")
    V = inputs.gaussian_rhs(621, n, 17)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="fp32_gram"))
    ref = gp.ky_matrix(okern(w), w.X) @ V.astype(np.float64)
    assert col_rel_err(out, ref).max() <= TOL


def test_gram_far_from_origin(mf):
    # Points away from the origin: the centring keeps |g|^2 small, so the Gram
    # branch runs and stays accurate although |u|^2 is about 1e3 (uncentred,
    # the form's error would be about 7e-5).
    banner("matvec fp32_gram rbf d=2 n=2000, X offset by 10")
    w = inputs.random_problem(622, 2000, 2, "rbf")
    X = (w.X + np.float32(10.0)).astype(np.float32)
    V = inputs.gaussian_rhs(623, 2000, 33)
    out = host(mf.kernel_matvec(mkern(w), dev(X), dev(V), precision="fp32_gram"))
    ref = gp.ky_matrix(okern(w), X) @ V.astype(np.float64)
    assert col_rel_err(out, ref).max() <= TOL


@pytest.mark.parametrize("t", [1, 33])
def test_gram_guard_falls_back(mf, t):
    # l = 0.02 on [0, 1]^2: max |g|^2 is about 900, far above the bound, so
    # every block takes the direct-difference branch; the result must still
    # meet the FP32 bar (the Gram branch would not).
    banner(f"matvec fp32_gram guard: rbf d=2 l=0.02 n=4000 t={t}")
    w = inputs.random_problem(624, 4000, 2, "rbf", lengthscale=0.02)
    V = inputs.gaussian_rhs(625, 4000, t)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="fp32_gram"))
    ref = gp.ky_matrix(okern(w), w.X) @ V.astype(np.float64)
    assert col_rel_err(out, ref).max() <= TOL


@pytest.mark.parametrize("t", [1, 33])
def test_gram_near_its_bound(mf, t):
    # l = 0.076 on [0, 1]^2: max |g|^2 is about 60, just under the bound of 62,
    # where the form's cancellation is largest: the Gram branch runs (the
    # result differs from the direct form's) and still meets the FP32 bar.
    banner(f"matvec fp32_gram near the guard: rbf d=2 l=0.076 n=4000 t={t}")
    w = inputs.random_problem(640, 4000, 2, "rbf", lengthscale=0.076)
    c = np.sqrt(np.log2(np.e) / 2)
    u = w.X.astype(np.float64) * c / 0.076
    g2 = ((u - u.mean(axis=0)) ** 2).sum(axis=1).max()
    assert 50.0 <= g2 <= 64.0, g2
    V = inputs.gaussian_rhs(641, 4000, t)
    k = mkern(w)
    out = host(mf.kernel_matvec(k, dev(w.X), dev(V), precision="fp32_gram"))
    direct = host(mf.kernel_matvec(k, dev(w.X), dev(V), precision="fp32_direct"))
    assert not np.array_equal(out, direct)
    ref = gp.ky_matrix(okern(w), w.X) @ V.astype(np.float64)
    err = col_rel_err(out, ref)
    print(f"max|g|^2 = {g2:.1f}: Gram-form column errors up to {err.max():.2e}")
    assert err.max() <= TOL


def _max_norm(X, lengthscale):
    u = X.astype(np.float64) * np.sqrt(np.log2(np.e) / 2) / np.asarray(lengthscale, dtype=np.float64)
    return float(((u - u.mean(axis=0)) ** 2).sum(axis=1).max())


@pytest.mark.parametrize("d,ls,t", [(2, 0.05, 1), (2, 0.05, 17), (1, 0.035, 33), (4, 0.07, 33),
                                    (6, 0.11, 1), (8, 0.12, 17)])
def test_gram_above_its_bound_runs_direct_differences(mf, d, ls, t):
    # 62 < max |g|^2 <= 160 (d = 2, l = 0.05 is the rbf500k geometry, about
    # 144): the factors would leave binary32, so the launch runs the direct
    # differences and meets the FP32 bar.
    banner(f"matvec fp32_gram above the bound: rbf d={d} l={ls} n=4000 t={t}")
    n = 3000 if d >= 7 else 4000
    w = inputs.random_problem((650 if d < 7 else 670) + d, n, d, "rbf", lengthscale=ls)
    g2 = _max_norm(w.X, ls)
    assert 62.0 < g2 <= 160.0, g2
    V = inputs.gaussian_rhs(660 + t, n, t)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="fp32_gram"))
    ref = gp.ky_matrix(okern(w), w.X) @ V.astype(np.float64)
    assert col_rel_err(out, ref).max() <= TOL


def test_gram_symmetric_operator(mf):
    # K~ is symmetric in the Gram form: u^T (K~ v) = v^T (K~ u) up to the
    # FP32 accumulation of the two products.
    banner("matvec fp32_gram symmetry u^T K v = v^T K u, n=4096")
    w = inputs.random_problem(626, 4096, 4, "rbf", ard=True)
    U = inputs.gaussian_rhs(627, 4096, 1)
    Vv = inputs.gaussian_rhs(628, 4096, 1)
    k = mkern(w)
    ku = host(mf.kernel_matvec(k, dev(w.X), dev(U), precision="fp32_gram")).astype(np.float64)
    kv = host(mf.kernel_matvec(k, dev(w.X), dev(Vv), precision="fp32_gram")).astype(np.float64)
    a = float(U[:, 0] @ kv.reshape(-1))
    b = float(Vv[:, 0] @ ku.reshape(-1))
    scale = float(np.abs(U[:, 0]) @ (gp.ky_matrix(okern(w), w.X) @ np.abs(Vv[:, 0])))
    assert abs(a - b) <= 1e-6 * scale


def test_gram_is_the_fp32_default_at_large_n(mf):
    # n >= 32768: MFGP_FP32 takes the Gram form for RBF; same result as
    # forcing it, bitwise, and within the bar of the direct form.
    banner("matvec rbf100k n=40000 t=33: fp32 == fp32_gram, vs fp32_direct")
    w = inputs.rbf100k(n=40000, probes=32)
    V = np.concatenate([w.y[:, None], w.Z], axis=1)
    k = mkern(w)
    a = host(mf.kernel_matvec(k, dev(w.X), dev(V), precision="fp32"))
    b = host(mf.kernel_matvec(k, dev(w.X), dev(V), precision="fp32_gram"))
    c = host(mf.kernel_matvec(k, dev(w.X), dev(V), precision="fp32_direct"))
    assert np.array_equal(a, b)
    assert col_rel_err(a, c.astype(np.float64)).max() <= TOL
    rows = np.random.default_rng(9).choice(w.n, size=512, replace=False)
    ref = gp.ky_matvec_rows(okern(w), w.X, V, rows)
    assert col_rel_err(a[rows], ref).max() <= TOL


def test_gram_cg_solve_exact1k(mf):
    # CG with the Gram operator, refined against the direct-difference FP64
    # residual: the same 1e-6 bar and the same solution.
    banner("cg_solve exact1k fp32_gram vs Cholesky")
    w = inputs.exact1k(probes=8)
    B = np.concatenate([w.y[:, None], w.Z], axis=1)
    x, info, _, st = mf.cg_solve(mkern(w), dev(w.X), dev(B), tol=1e-6, precision="fp32_gram")
    assert st == mf.OK, info
    assert max(i["rel_resid_true"] for i in info) <= 1e-6
    assert col_rel_err(host(x), gp.solve(okern(w), w.X, B)).max() <= 1e-4


# ---------------------------------------------------------------- bf16 forms
# n >= 32768 square RBF products of the bf16 forms take the same Gram form
# (distances on v_mfma_f32_32x32x2_f32, entries then split into bf16 pieces).
# Bars as for the direct-difference bf16 forms: x3 the FP32 bar, x2 3e-5, x1
# the bf16 bound 1e-2 (its floor is ~1e-3).
BF16_BARS = {"bf16x1": 1e-2, "bf16x2": 3e-5, "bf16x3": 1e-5}


@pytest.mark.parametrize("form", ["bf16x1", "bf16x2", "bf16x3"])
@pytest.mark.parametrize("t", [17, 33, 64, 65])
def test_gram_bf16_forms_sampled_rows(mf, form, t):
    # n = 40003: a ragged last 32-j distance tile and row block
    banner(f"matvec {form} Gram form rbf d=4 n=40003 t={t}, 384 sampled rows")
    w = inputs.random_problem(630, 40003, 4, "rbf", ard=True)
    V = inputs.gaussian_rhs(631 + t, 40003, t)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision=form))
    rows = np.random.default_rng(632).choice(w.n, size=384, replace=False)
    ref = gp.ky_matvec_rows(okern(w), w.X, V, rows)
    err = col_rel_err(out[rows], ref).max()
    print(f"{form} t={t}: max column error {err:.2e}")
    assert err <= BF16_BARS[form]
    assert np.isfinite(out).all()


@pytest.mark.parametrize("d", [1, 6])
def test_gram_bf16_dims(mf, d):
    # d = 1: one distance MFMA of two (one zero) dims; d = 6: four (DG = 8)
    banner(f"matvec bf16x3 Gram form rbf d={d} n=33000 t=33")
    w = inputs.random_problem(633 + d, 33000, d, "rbf", ard=True)
    V = inputs.gaussian_rhs(634, 33000, 33)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="bf16x3"))
    rows = np.random.default_rng(635).choice(w.n, size=256, replace=False)
    assert col_rel_err(out[rows], gp.ky_matvec_rows(okern(w), w.X, V, rows)).max() <= 1e-5


def test_gram_bf16_guard_falls_back(mf):
    # l = 0.02 on [0, 1]^2: max |g|^2 ~ 900, every block takes the direct
    # branch on the permuted fragments; x3 must still meet the FP32 bar
    banner("matvec bf16x3 Gram guard: rbf d=2 l=0.02 n=36000 t=33")
    w = inputs.random_problem(636, 36000, 2, "rbf", lengthscale=0.02)
    V = inputs.gaussian_rhs(637, 36000, 33)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="bf16x3"))
    rows = np.random.default_rng(638).choice(w.n, size=256, replace=False)
    assert col_rel_err(out[rows], gp.ky_matvec_rows(okern(w), w.X, V, rows)).max() <= 1e-5
