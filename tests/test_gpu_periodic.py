"""The periodic kernel family on the HIP path against the FP64 oracle.

The library evaluates k = s2 exp(-sum_k 2 sin^2(pi (x_k - x'_k) / p) / l_k^2)
as RBF on the 2d circle features (cos, sin)(2 pi x_k / p) / l_k, so every
product form of RBF runs on it; the gradient adds d/dp from its own adjoint
term.  The oracle evaluates the sine form directly (oracle/gp.py), so these
tests also check the feature identity, the phase reduction (inputs span
several periods) and the gradient order [l.., p, s2, sigma^2].  Bars: those
of the stationary families (1e-5 per-column FP32 products, 1e-6 CG residual,
1e-4 means and variances, 1e-3 gradients).
"""

import math

import numpy as np
import pytest

from oracle import gp, krylov, precond, variance
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, col_rel_err, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


def problem(seed, n, d, ard=True, period=0.45, noise=0.05, span=(-1.0, 2.0)):
    """Inputs spanning several periods, ARD lengthscales in [0.4, 1.2]."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(span[0], span[1], (n, d)).astype(np.float32)
    ls = [float(v) for v in rng.uniform(0.4, 1.2, d)] if ard else 0.7
    y = (np.sin(2 * np.pi * X / period).sum(axis=1) + 0.1 * rng.standard_normal(n)).astype(np.float32)
    ok = gp.Kern("periodic", ls, 1.3, noise, period=period)
    return X, y, ok


def mk(mf, ok):
    ls = ok.lengthscale
    ls = [float(v) for v in ls] if np.ndim(ls) == 1 else float(ls)
    return mf.Kernel("periodic", ls, ok.outputscale, ok.noise, period=ok.period)


def grad_ok(g, ref):
    g, ref = np.asarray(g), np.asarray(ref)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    comp = np.all(np.abs(g - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))
    return rel <= 1e-3 and comp, rel


@pytest.mark.parametrize("precision", ["fp32", "fp32_valu", "fp32_direct", "fp32_gram", "bf16x3"])
@pytest.mark.parametrize("d,t", [(1, 1), (2, 17), (4, 33)])
def test_matvec_vs_oracle(mf, precision, d, t):
    banner(f"periodic matvec n=1537 d={d} t={t} {precision}")
    X, _, ok = problem(900 + d, 1537, d)
    V = np.random.default_rng(901).standard_normal((1537, t)).astype(np.float32)
    out = mf.kernel_matvec(mk(mf, ok), dev(X), dev(V), precision=precision)
    ref = gp.ky_matvec(ok, X.astype(np.float64), V.astype(np.float64))
    err = col_rel_err(host(out), ref).max()
    print(f"max per-column relative error {err:.2e}")
    assert err <= 1e-5


def test_matvec_shared_lengthscale_and_short_period(mf):
    # many periods inside the data range (p = 0.05 over [0, 3]) and one shared l
    banner("periodic matvec n=700 d=3 shared l, p=0.05")
    X, _, ok = problem(905, 700, 3, ard=False, period=0.05, span=(0.0, 3.0))
    V = np.random.default_rng(906).standard_normal((700, 5)).astype(np.float32)
    out = mf.kernel_matvec(mk(mf, ok), dev(X), dev(V))
    ref = gp.ky_matvec(ok, X.astype(np.float64), V.astype(np.float64))
    assert col_rel_err(host(out), ref).max() <= 1e-5


def test_cg_and_predict_mean(mf):
    banner("periodic CG solve + predictive mean n=1200 d=2 m=301")
    X, y, ok = problem(910, 1200, 2, noise=0.1)
    k = mk(mf, ok)
    x, info, _, st = mf.cg_solve(k, dev(X), dev(y), tol=1e-6)
    assert st == mf.OK, info
    assert info[0]["rel_resid_true"] <= 1e-6
    Xd = X.astype(np.float64)
    alpha = gp.solve(ok, Xd, y.astype(np.float64))
    assert np.linalg.norm(host(x) - alpha) / np.linalg.norm(alpha) <= 1e-4
    Xs = np.random.default_rng(911).uniform(-1.5, 2.5, (301, 2)).astype(np.float32)
    mu = mf.predict_mean(k, dev(X), dev(Xs), x.float())
    ref = gp.predict_mean(ok, Xd, Xs.astype(np.float64), alpha)
    assert np.abs(host(mu) - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("d,ard", [(1, False), (2, True), (3, True), (4, False)])
def test_adjoint_vs_oracle(mf, d, ard):
    # sum_c w_c A_c^T dK/dtheta B_c for [l.., p, s2, sigma^2]: the period term is
    # the new adjoint sum; the lengthscale terms pair the two circle features
    banner(f"periodic adjoint n=900 d={d} ard={ard} t=3")
    X, _, ok = problem(920 + d, 900, d, ard=ard)
    rng = np.random.default_rng(921)
    A = rng.standard_normal((900, 3)).astype(np.float32)
    B = rng.standard_normal((900, 3)).astype(np.float32)
    colw = [0.5, -0.25, 1.5]
    g = np.array(mf.kernel_adjoint(mk(mf, ok), dev(X), dev(A), dev(B), colw))
    ref = gp.adjoint_bilinear(ok, X, A, B, colw)
    assert len(g) == ok.n_params(d)
    print("adjoint", g, ref)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-4
    assert np.all(np.abs(g - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))


def test_mll_same_probe(mf):
    banner("periodic mll+grad n=1000 d=2 ARD p=8 vs same-probe oracle")
    X, y, ok = problem(930, 1000, 2, noise=0.08)
    Z = inputs.rademacher(np.random.default_rng(931), 1000, 8)
    r = mf.mll_and_grad(mk(mf, ok), dev(X), dev(y), Z=dev(Z), tol=1e-6)
    assert r["status"] == mf.OK, r["info"]
    Xd, yd = X.astype(np.float64), y.astype(np.float64)
    ld = float(krylov.quadform_log(gp.ky_matrix(ok, Xd), Z).mean())
    alpha = gp.solve(ok, Xd, yd)
    mll = -0.5 * (float(yd @ alpha) + ld + len(yd) * math.log(2 * math.pi))
    assert r["logdet"] == pytest.approx(ld, rel=1e-4)
    assert r["mll"] == pytest.approx(mll, rel=1e-4)
    ok_, rel = grad_ok(r["grad"], gp.same_probe_grad(ok, Xd, yd, Z))
    assert ok_, (r["grad"], rel)


@pytest.mark.parametrize("ard", [False, True])
def test_mll_exact_mode_vs_cholesky_and_fd(mf, ard):
    # probes sqrt(N) e_c make the log-det and the trace exact: the gradient,
    # d/dp included, is checked against the exact one and central differences
    banner(f"periodic exact-mode mll+grad n=200 d=2 ard={ard}")
    n = 200
    X, y, ok = problem(940, n, 2, ard=ard, noise=0.05)
    Z = (math.sqrt(n) * np.eye(n)).astype(np.float32)
    r = mf.mll_and_grad(mk(mf, ok), dev(X), dev(y), Z=dev(Z), tol=1e-7)
    assert r["status"] == mf.OK
    Xd, yd = X.astype(np.float64), y.astype(np.float64)
    assert r["logdet"] == pytest.approx(gp.logdet(ok, Xd), rel=1e-4)
    assert r["mll"] == pytest.approx(gp.mll(ok, Xd, yd), rel=1e-4)
    ok_, rel = grad_ok(r["grad"], gp.mll_grad(ok, Xd, yd))
    assert ok_, (r["grad"], rel)
    th = ok.params(2)
    fd = []
    for q in range(len(th)):
        h = 1e-5 * th[q]
        tp, tm = th.copy(), th.copy()
        tp[q] += h
        tm[q] -= h
        fd.append((gp.mll(ok.with_params(tp), Xd, yd) - gp.mll(ok.with_params(tm), Xd, yd)) / (2 * h))
    ok_, rel = grad_ok(r["grad"], fd)
    assert ok_, (r["grad"], fd, rel)


def test_variance_same_probe(mf):
    banner("periodic predict_variance n=900 m=150 p=12 vs same-probe oracle")
    X, _, ok = problem(950, 900, 2, noise=0.1)
    Xs = np.random.default_rng(951).uniform(-1.5, 2.5, (150, 2)).astype(np.float32)
    Z = inputs.rademacher(np.random.default_rng(952), 150, 12)
    var, info, st = mf.predict_variance(mk(mf, ok), dev(X), dev(Xs), Z=dev(Z), tol=1e-6)
    assert st == mf.OK, info
    ref = variance.same_probe_variance(ok, X, Xs, Z)
    assert np.abs(host(var).astype(np.float64) - ref).max() <= 1e-4 * ok.outputscale


def test_pivoted_cholesky_and_pcg(mf):
    banner("periodic pivoted Cholesky rank 24 + PCG n=800 d=2")
    X, y, ok = problem(960, 800, 2, noise=0.05)
    k = mk(mf, ok)
    L, piv = mf.pivoted_cholesky(k, dev(X), 24)
    Lo, pivo = precond.pivoted_cholesky(ok, X, 24)
    np.testing.assert_array_equal(host(piv), pivo)
    assert np.abs(host(L).T - Lo).max() <= 2e-5 * np.sqrt(ok.outputscale)
    x, info, _, st = mf.precond_cg_solve(k, dev(X), dev(y), L, tol=1e-6)
    assert st == mf.OK, info
    alpha = gp.solve(ok, X.astype(np.float64), y.astype(np.float64))
    assert np.linalg.norm(host(x) - alpha) / np.linalg.norm(alpha) <= 1e-4


def test_gram_guard_large_features(mf):
    # short lengthscales make |g|^2 > 64: the Gram launch must take direct
    # differences and still meet the FP32 bar
    banner("periodic fp32_gram with |g|^2 > 64 (l = 0.08), n=1100 d=2")
    X, _, ok = problem(970, 1100, 2, ard=False)
    ok = gp.Kern("periodic", 0.08, 1.3, 0.05, period=0.45)
    V = np.random.default_rng(971).standard_normal((1100, 17)).astype(np.float32)
    out = mf.kernel_matvec(mk(mf, ok), dev(X), dev(V), precision="fp32_gram")
    ref = gp.ky_matvec(ok, X.astype(np.float64), V.astype(np.float64))
    assert col_rel_err(host(out), ref).max() <= 1e-5


def test_periodic_default_fp32_at_gram_size(mf):
    # n >= 32768: the default FP32 product takes the Gram form with DG = 8
    # (d = 4, 8 circle features); sampled rows against the oracle
    banner("periodic d=4 default fp32 n=40003 t=33 (Gram form, 8 features), sampled rows")
    X, _, ok = problem(990, 40003, 4, ard=True)
    V = np.random.default_rng(991).standard_normal((40003, 33)).astype(np.float32)
    out = host(mf.kernel_matvec(mk(mf, ok), dev(X), dev(V)))
    rows = np.random.default_rng(992).choice(40003, 200, replace=False)
    ref = gp.ky_matvec_rows(ok, X.astype(np.float64), V.astype(np.float64), rows)
    err = np.linalg.norm(out[rows] - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print(f"sampled-row relative error {err.max():.2e}")
    assert err.max() <= 1e-5
