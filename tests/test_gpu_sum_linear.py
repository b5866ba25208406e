"""Kernel sums and the Linear family on the HIP path against the FP64 oracle.

The sum tested throughout is the paper's composition example widened by a
linear term: Scale(RBF, ARD) + Scale(Periodic) + Scale(Linear) (Sec. 3
"Kernels"), evaluated term by term (each stationary term through the product
form of the precision, the linear term as s2 X (X^T V) in FP64).  The oracle
forms the dense sum (oracle/gp.py SumKern).  Bars: those of the single
families (1e-5 per-column FP32 products, 1e-6 CG residual, 1e-4 means,
variances and log-dets, 1e-3 gradients).
"""

import math

import numpy as np
import pytest

from oracle import gp, krylov, variance
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, col_rel_err, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


def data(seed, n, d=2, span=(-1.0, 2.0)):
    rng = np.random.default_rng(seed)
    X = rng.uniform(span[0], span[1], (n, d)).astype(np.float32)
    y = (X @ rng.standard_normal(d) + np.sin(2 * np.pi * X[:, 0] / 0.45) + 0.1 * rng.standard_normal(n))
    return X, y.astype(np.float32)


def sum_kernels(mf, noise=0.05, d=2):
    ls = [0.4, 0.9, 0.6, 0.5][:d]
    o = gp.SumKern([gp.Kern("rbf", np.array(ls), 1.1, 0.0),
                    gp.Kern("periodic", 0.7, 0.6, 0.0, period=0.45),
                    gp.Kern("linear", 1.0, 0.3, 0.0)], noise)
    k = (mf.Kernel("rbf", ls, 1.1, noise) + mf.Kernel("periodic", 0.7, 0.6, period=0.45)
         + mf.Kernel("linear", 1.0, 0.3))
    return o, k


def grad_ok(g, ref):
    g, ref = np.asarray(g), np.asarray(ref)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    comp = np.all(np.abs(g - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))
    return rel <= 1e-3 and comp, rel


@pytest.mark.parametrize("precision", ["fp32", "fp32_valu", "fp32_gram", "bf16x3"])
@pytest.mark.parametrize("t", [1, 17, 33])
def test_sum_matvec_vs_oracle(mf, precision, t):
    banner(f"sum rbf+periodic+linear matvec n=1537 t={t} {precision}")
    X, _ = data(1000 + t, 1537)
    o, k = sum_kernels(mf)
    V = np.random.default_rng(1001).standard_normal((1537, t)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V), precision=precision)
    ref = gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))
    err = col_rel_err(host(out), ref).max()
    print(f"max per-column relative error {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("d,t", [(1, 1), (3, 5), (8, 33)])
def test_linear_matvec_vs_oracle(mf, d, t):
    banner(f"linear matvec n=2049 d={d} t={t}")
    X, _ = data(1010 + d, 2049, d)
    o = gp.Kern("linear", 1.0, 0.7, 0.1)
    V = np.random.default_rng(1011).standard_normal((2049, t)).astype(np.float32)
    out = mf.kernel_matvec(mf.Kernel("linear", 1.0, 0.7, 0.1), dev(X), dev(V))
    ref = gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))
    assert col_rel_err(host(out), ref).max() <= 1e-5


def test_sum_residual_vs_oracle(mf):
    banner("sum residual B - K_y X (FP64 accumulation) n=900 t=3")
    X, _ = data(1020, 900)
    o, k = sum_kernels(mf)
    rng = np.random.default_rng(1021)
    B = rng.standard_normal((900, 3)).astype(np.float32)
    Xs = rng.standard_normal((900, 3))
    R, rel = mf.residual(k, dev(X), dev(B), dev(Xs))
    ref = B.astype(np.float64) - gp.ky_matvec(o, X.astype(np.float64), Xs)
    err = np.abs(host(R) - ref).max() / np.abs(ref).max()
    print(f"max |R - oracle| / max |R| = {err:.2e}")
    assert err <= 1e-5


def test_sum_cg_and_predict_mean(mf):
    banner("sum CG solve + predictive mean n=1200 m=257")
    X, y = data(1030, 1200)
    o, k = sum_kernels(mf, noise=0.1)
    x, info, _, st = mf.cg_solve(k, dev(X), dev(y), tol=1e-6)
    assert st == mf.OK, info
    assert info[0]["rel_resid_true"] <= 1e-6
    Xd = X.astype(np.float64)
    alpha = gp.solve(o, Xd, y.astype(np.float64))
    assert np.linalg.norm(host(x) - alpha) / np.linalg.norm(alpha) <= 1e-4
    Xs = np.random.default_rng(1031).uniform(-1.5, 2.5, (257, 2)).astype(np.float32)
    mu = mf.predict_mean(k, dev(X), dev(Xs), x.float())
    ref = gp.predict_mean(o, Xd, Xs.astype(np.float64), alpha)
    assert np.abs(host(mu) - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


def test_linear_cg_predict_is_ridge_regression(mf):
    # a linear GP's mean is ridge regression; K is rank d, so CG ends in a few steps
    banner("linear CG + predictive mean n=3000 d=3")
    X, y = data(1040, 3000, 3)
    k = mf.Kernel("linear", 1.0, 1.3, 0.2)
    x, info, _, st = mf.cg_solve(k, dev(X), dev(y), tol=1e-6)
    assert st == mf.OK, info
    Xs = np.random.default_rng(1041).uniform(-2, 3, (100, 3)).astype(np.float32)
    mu = host(mf.predict_mean(k, dev(X), dev(Xs), x.float())).astype(np.float64)
    Xd = X.astype(np.float64)
    ref = gp.predict_mean(gp.Kern("linear", 1.0, 1.3, 0.2), Xd, Xs.astype(np.float64),
                          gp.solve(gp.Kern("linear", 1.0, 1.3, 0.2), Xd, y.astype(np.float64)))
    assert np.abs(mu - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("which", ["sum", "linear", "rbf+matern32"])
def test_adjoint_vs_oracle(mf, which):
    banner(f"adjoint {which} n=800 t=3")
    X, _ = data(1050, 800)
    if which == "sum":
        o, k = sum_kernels(mf)
    elif which == "linear":
        o, k = gp.Kern("linear", 1.0, 0.8, 0.05), mf.Kernel("linear", 1.0, 0.8, 0.05)
    else:
        o = gp.SumKern([gp.Kern("rbf", 0.3, 0.9, 0.0), gp.Kern("matern32", np.array([0.5, 1.2]), 0.4, 0.0)], 0.05)
        k = mf.Kernel("rbf", 0.3, 0.9, 0.05) + mf.Kernel("matern32", [0.5, 1.2], 0.4)
    rng = np.random.default_rng(1051)
    A = rng.standard_normal((800, 3)).astype(np.float32)
    B = rng.standard_normal((800, 3)).astype(np.float32)
    colw = [0.5, -0.25, 1.5]
    g = np.array(mf.kernel_adjoint(k, dev(X), dev(A), dev(B), colw))
    ref = gp.adjoint_bilinear(o, X, A, B, colw)
    assert len(g) == o.n_params(2)
    print("adjoint", g, ref)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-4
    assert np.all(np.abs(g - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))


def test_sum_mll_same_probe(mf):
    banner("sum mll+grad n=1000 p=8 vs same-probe oracle")
    X, y = data(1060, 1000)
    o, k = sum_kernels(mf, noise=0.08)
    Z = inputs.rademacher(np.random.default_rng(1061), 1000, 8)
    r = mf.mll_and_grad(k, dev(X), dev(y), Z=dev(Z), tol=1e-6)
    assert r["status"] == mf.OK, r["info"]
    Xd, yd = X.astype(np.float64), y.astype(np.float64)
    ld = float(krylov.quadform_log(gp.ky_matrix(o, Xd), Z).mean())
    alpha = gp.solve(o, Xd, yd)
    mll = -0.5 * (float(yd @ alpha) + ld + len(yd) * math.log(2 * math.pi))
    assert r["logdet"] == pytest.approx(ld, rel=1e-4)
    assert r["mll"] == pytest.approx(mll, rel=1e-4)
    ok_, rel = grad_ok(r["grad"], gp.same_probe_grad(o, Xd, yd, Z))
    assert ok_, (r["grad"], rel)


@pytest.mark.parametrize("which", ["sum", "linear"])
def test_mll_exact_mode_vs_cholesky_and_fd(mf, which):
    banner(f"{which} exact-mode mll+grad n=200")
    n = 200
    X, y = data(1070, n)
    if which == "sum":
        o, k = sum_kernels(mf, noise=0.05)
    else:
        o, k = gp.Kern("linear", 1.0, 0.8, 0.05), mf.Kernel("linear", 1.0, 0.8, 0.05)
    Z = (math.sqrt(n) * np.eye(n)).astype(np.float32)
    r = mf.mll_and_grad(k, dev(X), dev(y), Z=dev(Z), tol=1e-7)
    assert r["status"] == mf.OK
    Xd, yd = X.astype(np.float64), y.astype(np.float64)
    assert r["logdet"] == pytest.approx(gp.logdet(o, Xd), rel=1e-4)
    assert r["mll"] == pytest.approx(gp.mll(o, Xd, yd), rel=1e-4)
    ok_, rel = grad_ok(r["grad"], gp.mll_grad(o, Xd, yd))
    assert ok_, (r["grad"], rel)
    th = o.params(2)
    fd = []
    for q in range(len(th)):
        h = 1e-5 * th[q]
        tp, tm = th.copy(), th.copy()
        tp[q] += h
        tm[q] -= h
        fd.append((gp.mll(o.with_params(tp), Xd, yd) - gp.mll(o.with_params(tm), Xd, yd)) / (2 * h))
    ok_, rel = grad_ok(r["grad"], fd)
    assert ok_, (r["grad"], fd, rel)


def test_sum_variance_same_probe(mf):
    # the prior variance of the sum includes the linear term's s2 |x*|^2
    banner("sum predict_variance n=900 m=150 p=12 vs same-probe oracle")
    X, _ = data(1080, 900)
    o, k = sum_kernels(mf, noise=0.1)
    Xs = np.random.default_rng(1081).uniform(-1.5, 2.5, (150, 2)).astype(np.float32)
    Z = inputs.rademacher(np.random.default_rng(1082), 150, 12)
    var, info, st = mf.predict_variance(k, dev(X), dev(Xs), Z=dev(Z), tol=1e-6)
    assert st == mf.OK, info
    ref = variance.same_probe_variance(o, X, Xs, Z)
    prior = variance.prior_variance(o, Xs)
    assert np.abs(host(var).astype(np.float64) - ref).max() <= 1e-4 * prior.max()


def test_sum_of_two_gram_terms_at_gram_size(mf):
    # two RBF terms at n >= 32768: both take the Gram form in the default FP32
    banner("sum rbf(l=0.3)+rbf(l=0.8) matvec n=40003 d=4 t=33, sampled rows")
    w = inputs.random_problem(1090, 40003, 4, "rbf")
    o = gp.SumKern([gp.Kern("rbf", 0.3, 1.0, 0.0), gp.Kern("rbf", 0.8, 0.5, 0.0)], 0.02)
    k = mf.Kernel("rbf", 0.3, 1.0, 0.02) + mf.Kernel("rbf", 0.8, 0.5)
    V = np.random.default_rng(1091).standard_normal((40003, 33)).astype(np.float32)
    out = host(mf.kernel_matvec(k, dev(w.X), dev(V)))
    rows = np.random.default_rng(1092).choice(40003, 300, replace=False)
    ref = gp.ky_matvec_rows(o, w.X.astype(np.float64), V.astype(np.float64), rows)
    err = np.linalg.norm(out[rows] - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= 1e-5


def test_linear_head_sum_matvec_and_cg(mf):
    # the linear term first: it writes the product with the noise, the
    # Matern term adds into it; CG on the sum reaches the 1e-6 residual
    banner("sum linear+matern52 (linear head) matvec and CG n=1100 d=3")
    X, y = data(1100, 1100, 3)
    o = gp.SumKern([gp.Kern("linear", 1.0, 0.2, 0.0), gp.Kern("matern52", np.array([0.5, 0.8, 1.1]), 1.2, 0.0)],
                   0.07)
    k = mf.Kernel("linear", 1.0, 0.2, 0.07) + mf.Kernel("matern52", [0.5, 0.8, 1.1], 1.2)
    V = np.random.default_rng(1101).standard_normal((1100, 17)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V))
    Xd = X.astype(np.float64)
    assert col_rel_err(host(out), gp.ky_matvec(o, Xd, V.astype(np.float64))).max() <= 1e-5
    x, info, _, st = mf.cg_solve(k, dev(X), dev(y), tol=1e-6)
    assert st == mf.OK, info
    alpha = gp.solve(o, Xd, y.astype(np.float64))
    assert np.linalg.norm(host(x) - alpha) / np.linalg.norm(alpha) <= 1e-4


def two_term(mf, l_rbf=0.4, noise=0.05):
    o = gp.SumKern([gp.Kern("rbf", np.array([l_rbf, 2 * l_rbf]), 1.1, 0.0),
                    gp.Kern("periodic", 0.7, 0.6, 0.0, period=0.45)], noise)
    k = mf.Kernel("rbf", [l_rbf, 2 * l_rbf], 1.1, noise) + mf.Kernel("periodic", 0.7, 0.6, period=0.45)
    return o, k


@pytest.mark.parametrize("t", [1, 17, 33])
def test_fused_two_term_gram_matvec(mf, t):
    # two RBF-class terms in the Gram form run as one fused sweep (one contraction)
    banner(f"fused two-term sum rbf+periodic fp32_gram n=1537 t={t}")
    X, _ = data(1600 + t, 1537)
    o, k = two_term(mf)
    V = np.random.default_rng(1601).standard_normal((1537, t)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V), precision="fp32_gram")
    ref = gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))
    err = col_rel_err(host(out), ref).max()
    print(f"max per-column relative error {err:.2e}")
    assert err <= 1e-5


def test_fused_two_term_direct_fallback(mf):
    # short RBF lengthscales push max |g|^2 past the Gram bound: the fused
    # sweep takes direct differences for both terms
    banner("fused two-term sum with |g|^2 > 64 (direct differences), n=1100 t=17")
    X, _ = data(1610, 1100)
    o, k = two_term(mf, l_rbf=0.05)
    V = np.random.default_rng(1611).standard_normal((1100, 17)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V), precision="fp32_gram")
    ref = gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))
    assert col_rel_err(host(out), ref).max() <= 1e-5


def test_fused_two_term_mll(mf):
    banner("fused two-term sum mll+grad fp32_gram n=1000 p=8 vs same-probe oracle")
    X, y = data(1620, 1000)
    o, k = two_term(mf, noise=0.08)
    Z = inputs.rademacher(np.random.default_rng(1621), 1000, 8)
    r = mf.mll_and_grad(k, dev(X), dev(y), Z=dev(Z), tol=1e-6, precision="fp32_gram")
    assert r["status"] == mf.OK, r["info"]
    Xd, yd = X.astype(np.float64), y.astype(np.float64)
    ld = float(krylov.quadform_log(gp.ky_matrix(o, Xd), Z).mean())
    assert r["logdet"] == pytest.approx(ld, rel=1e-4)
    ok_, rel = grad_ok(r["grad"], gp.same_probe_grad(o, Xd, yd, Z))
    assert ok_, (r["grad"], rel)


@pytest.mark.parametrize("case", ["periodic6+rbf3", "periodic8+periodic8"])
def test_fused_two_term_operand_widths(mf, case):
    # the fused sweep's instances by the terms' operand widths: DG = 8 then 4
    # (6 circle features + 3 RBF features) and DG = 8 for both (d = 4 circles)
    banner(f"fused two-term sum {case} fp32_gram n=1300 t=33")
    if case == "periodic6+rbf3":
        d = 3
        o = gp.SumKern([gp.Kern("periodic", np.array([0.8, 1.1, 0.9]), 0.7, 0.0, period=0.5),
                        gp.Kern("rbf", 0.6, 1.2, 0.0)], 0.05)
        k = mf.Kernel("periodic", [0.8, 1.1, 0.9], 0.7, 0.05, period=0.5) + mf.Kernel("rbf", 0.6, 1.2)
    else:
        d = 4
        o = gp.SumKern([gp.Kern("periodic", 1.0, 0.9, 0.0, period=0.45),
                        gp.Kern("periodic", np.array([1.2, 0.9, 1.4, 1.1]), 0.4, 0.0, period=1.3)], 0.05)
        k = mf.Kernel("periodic", 1.0, 0.9, 0.05, period=0.45) + \
            mf.Kernel("periodic", [1.2, 0.9, 1.4, 1.1], 0.4, period=1.3)
    X, _ = data(1630 + d, 1300, d)
    V = np.random.default_rng(1631).standard_normal((1300, 33)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V), precision="fp32_gram")
    ref = gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))
    err = col_rel_err(host(out), ref).max()
    print(f"max per-column relative error {err:.2e}")
    assert err <= 1e-5


def test_four_term_sum_maximum(mf):
    # MFGP_MAX_TERMS terms of four different kinds: matvec and adjoint
    banner("sum of 4 terms (rbf, matern12, periodic, linear) n=900 t=5")
    X, _ = data(1700, 900, 2)
    o = gp.SumKern([gp.Kern("rbf", 0.4, 1.0, 0.0), gp.Kern("matern12", np.array([0.6, 0.9]), 0.5, 0.0),
                    gp.Kern("periodic", 0.7, 0.4, 0.0, period=0.45), gp.Kern("linear", 1.0, 0.2, 0.0)], 0.05)
    k = (mf.Kernel("rbf", 0.4, 1.0, 0.05) + mf.Kernel("matern12", [0.6, 0.9], 0.5)
         + mf.Kernel("periodic", 0.7, 0.4, period=0.45) + mf.Kernel("linear", 1.0, 0.2))
    V = np.random.default_rng(1701).standard_normal((900, 5)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V))
    assert col_rel_err(host(out), gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))).max() <= 1e-5
    A = np.random.default_rng(1702).standard_normal((900, 2)).astype(np.float32)
    B = np.random.default_rng(1703).standard_normal((900, 2)).astype(np.float32)
    g = np.array(mf.kernel_adjoint(k, dev(X), dev(A), dev(B), [1.0, -0.5]))
    ref = gp.adjoint_bilinear(o, X, A, B, [1.0, -0.5])
    assert len(g) == o.n_params(2) == 10      # [l, s2 | l1, l2, s2 | l, p, s2 | s2 | sigma^2]
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-4


@pytest.mark.parametrize("which", ["sum", "prod"])
def test_single_point_compositions(mf, which):
    banner(f"{which} with n = 1")
    X = np.array([[0.3, -0.2]], np.float32)
    V = np.array([[1.5, -2.0]], np.float32)
    if which == "sum":
        o, k = sum_kernels(mf)
    else:
        o = gp.ProdKern([gp.Kern("rbf", 0.5, 1.0, 0.0), gp.Kern("periodic", 0.7, 1.0, 0.0, period=0.45)], 1.3, 0.05)
        k = mf.Kernel("rbf", 0.5, 1.3, 0.05) * mf.Kernel("periodic", 0.7, period=0.45)
    out = host(mf.kernel_matvec(k, dev(X), dev(V)))
    np.testing.assert_allclose(out, gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64)), rtol=1e-6)


def test_fused_composite_full_size_sampled_rows(mf):
    # the composite leg's product: Scale(RBF) + Scale(Periodic) on the rbf100k
    # points (N = 1e5, d = 4, t = 33), the default FP32 launch (fused Gram
    # sweep), against the oracle on 256 sampled rows
    banner("fused rbf+periodic rbf100k full size t=33, 256 sampled rows")
    w = inputs.rbf100k()
    o = gp.SumKern([gp.Kern("rbf", w.lengthscale, w.outputscale, 0.0),
                    gp.Kern("periodic", 1.0, 0.5 * w.outputscale, 0.0, period=0.5)], w.noise)
    k = (mf.Kernel("rbf", w.lengthscale, w.outputscale, w.noise)
         + mf.Kernel("periodic", 1.0, 0.5 * w.outputscale, period=0.5))
    V = np.concatenate([w.y[:, None], w.Z], axis=1).astype(np.float32)
    out = host(mf.kernel_matvec(k, dev(w.X), dev(V)))
    rows = np.random.default_rng(1800).choice(w.n, 256, replace=False)
    ref = gp.ky_matvec_rows(o, w.X.astype(np.float64), V.astype(np.float64), rows)
    err = np.linalg.norm(out[rows] - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print(f"sampled-row relative error {err.max():.2e}")
    assert err.max() <= 1e-5
