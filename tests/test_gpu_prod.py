"""Kernel products on the HIP path against the FP64 oracle (oracle/gp.py ProdKern).

A product of RBF factors and at most one periodic factor is RBF with unit
lengthscales on the concatenated features (the periodic factor's circle
features first), so it runs every RBF product form; its gradient takes each
factor's lengthscales from the per-feature adjoint sums and the period from
the periodic adjoint term.  Bars as for the single families.
"""

import math

import numpy as np
import pytest

from oracle import gp, precond, variance
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, col_rel_err, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


def data(seed, n, d=2):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 2.0, (n, d)).astype(np.float32)
    y = (np.sin(2 * np.pi * X[:, 0] / 0.45) * np.exp(-0.3 * X[:, -1] ** 2) + 0.1 * rng.standard_normal(n))
    return X, y.astype(np.float32)


def rbf_per(mf, noise=0.05, s2=1.3):
    o = gp.ProdKern([gp.Kern("rbf", np.array([0.6, 1.4]), 1.0, 0.0),
                     gp.Kern("periodic", 0.8, 1.0, 0.0, period=0.45)], s2, noise)
    k = mf.Kernel("rbf", [0.6, 1.4], s2, noise) * mf.Kernel("periodic", 0.8, period=0.45)
    return o, k


def grad_ok(g, ref):
    g, ref = np.asarray(g), np.asarray(ref)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    comp = np.all(np.abs(g - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))
    return rel <= 1e-3 and comp, rel


@pytest.mark.parametrize("precision", ["fp32", "fp32_valu", "fp32_gram", "bf16x3"])
@pytest.mark.parametrize("t", [1, 33])
def test_product_matvec_vs_oracle(mf, precision, t):
    banner(f"rbf*periodic matvec n=1537 d=2 t={t} {precision}")
    X, _ = data(1200 + t, 1537)
    o, k = rbf_per(mf)
    V = np.random.default_rng(1201).standard_normal((1537, t)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V), precision=precision)
    ref = gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))
    assert col_rel_err(host(out), ref).max() <= 1e-5


def test_rbf_times_rbf_matvec(mf):
    banner("rbf*rbf matvec n=1100 d=4 (8 features) t=17")
    X, _ = data(1210, 1100, 4)
    o = gp.ProdKern([gp.Kern("rbf", np.array([0.5, 0.9, 1.3, 0.7]), 1.0, 0.0), gp.Kern("rbf", 0.8, 1.0, 0.0)],
                    0.9, 0.1)
    k = mf.Kernel("rbf", [0.5, 0.9, 1.3, 0.7], 0.9, 0.1) * mf.Kernel("rbf", 0.8)
    V = np.random.default_rng(1211).standard_normal((1100, 17)).astype(np.float32)
    out = mf.kernel_matvec(k, dev(X), dev(V))
    assert col_rel_err(host(out), gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))).max() <= 1e-5


@pytest.mark.parametrize("which", ["rbf*per d=2", "rbf*rbf*per d=1", "per*rbf*rbf*rbf d=1", "rbf*rbf d=2"])
def test_product_adjoint_vs_oracle(mf, which):
    banner(f"adjoint {which} n=800 t=3")
    if which == "rbf*per d=2":
        d = 2
        o, k = rbf_per(mf)
    elif which == "rbf*rbf*per d=1":
        d = 1
        o = gp.ProdKern([gp.Kern("rbf", 0.7, 1.0, 0.0), gp.Kern("rbf", 1.6, 1.0, 0.0),
                         gp.Kern("periodic", 0.9, 1.0, 0.0, period=0.3)], 0.8, 0.05)
        k = mf.Kernel("rbf", 0.7, 0.8, 0.05) * mf.Kernel("rbf", 1.6) * mf.Kernel("periodic", 0.9, period=0.3)
    elif which == "per*rbf*rbf*rbf d=1":
        d = 1
        o = gp.ProdKern([gp.Kern("periodic", [0.9], 1.0, 0.0, period=0.3), gp.Kern("rbf", 0.7, 1.0, 0.0),
                         gp.Kern("rbf", [1.6], 1.0, 0.0), gp.Kern("rbf", 2.5, 1.0, 0.0)], 0.8, 0.05)
        k = (mf.Kernel("periodic", [0.9], 0.8, 0.05, period=0.3) * mf.Kernel("rbf", 0.7)
             * mf.Kernel("rbf", [1.6]) * mf.Kernel("rbf", 2.5))
    else:
        d = 2
        o = gp.ProdKern([gp.Kern("rbf", np.array([0.6, 1.4]), 1.0, 0.0), gp.Kern("rbf", 0.9, 1.0, 0.0)], 1.1, 0.05)
        k = mf.Kernel("rbf", [0.6, 1.4], 1.1, 0.05) * mf.Kernel("rbf", 0.9)
    X, _ = data(1220, 800, d)
    rng = np.random.default_rng(1221)
    A = rng.standard_normal((800, 3)).astype(np.float32)
    B = rng.standard_normal((800, 3)).astype(np.float32)
    colw = [0.5, -0.25, 1.5]
    g = np.array(mf.kernel_adjoint(k, dev(X), dev(A), dev(B), colw))
    ref = gp.adjoint_bilinear(o, X, A, B, colw)
    assert len(g) == o.n_params(d)
    print("adjoint", g, ref)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-4
    assert np.all(np.abs(g - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))


@pytest.mark.parametrize("which", ["prod", "sum_with_prod"])
def test_mll_exact_mode_vs_cholesky_and_fd(mf, which):
    banner(f"{which} exact-mode mll+grad n=200 d=2")
    n = 200
    X, y = data(1230, n)
    o, k = rbf_per(mf, noise=0.05)
    if which == "sum_with_prod":
        o = gp.SumKern([o, gp.Kern("linear", 1.0, 0.3, 0.0)], 0.05)
        k = k + mf.Kernel("linear", 1.0, 0.3)
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


def test_sum_with_product_cg_predict_variance(mf):
    banner("rbf*periodic + matern52: CG, predictive mean and variance n=1000 m=120")
    X, y = data(1240, 1000)
    o, k = rbf_per(mf, noise=0.1)
    o = gp.SumKern([o, gp.Kern("matern52", 1.5, 0.5, 0.0)], 0.1)
    k = k + mf.Kernel("matern52", 1.5, 0.5)
    x, info, _, st = mf.cg_solve(k, dev(X), dev(y), tol=1e-6)
    assert st == mf.OK, info
    Xd = X.astype(np.float64)
    alpha = gp.solve(o, Xd, y.astype(np.float64))
    assert np.linalg.norm(host(x) - alpha) / np.linalg.norm(alpha) <= 1e-4
    Xs = np.random.default_rng(1241).uniform(-1.5, 2.5, (120, 2)).astype(np.float32)
    mu = mf.predict_mean(k, dev(X), dev(Xs), x.float())
    ref = gp.predict_mean(o, Xd, Xs.astype(np.float64), alpha)
    assert np.abs(host(mu) - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    Z = inputs.rademacher(np.random.default_rng(1242), 120, 8)
    var, _, st = mf.predict_variance(k, dev(X), dev(Xs), Z=dev(Z), tol=1e-6)
    assert st == mf.OK
    vref = variance.same_probe_variance(o, X, Xs, Z)
    assert np.abs(host(var).astype(np.float64) - vref).max() <= 1e-4 * 1.8


def test_product_pivoted_cholesky_and_pcg(mf):
    banner("rbf*periodic pivoted Cholesky rank 24 + PCG n=800")
    X, y = data(1250, 800)
    o, k = rbf_per(mf, noise=0.05)
    L, piv = mf.pivoted_cholesky(k, dev(X), 24)
    Lo, pivo = precond.pivoted_cholesky(o, X, 24)
    np.testing.assert_array_equal(host(piv), pivo)
    assert np.abs(host(L).T - Lo).max() <= 2e-5 * np.sqrt(o.outputscale)
    x, info, _, st = mf.precond_cg_solve(k, dev(X), dev(y), L, tol=1e-6)
    assert st == mf.OK, info
    alpha = gp.solve(o, X.astype(np.float64), y.astype(np.float64))
    assert np.linalg.norm(host(x) - alpha) / np.linalg.norm(alpha) <= 1e-4


# ---------------------------------------------------------------- general products
# Products with Matern or Linear factors run the general-product sweeps
# (one exp2 per entry over all factors, FP32 entries on the VALU).

def general(mf, which):
    """(oracle kernel, library kernel, d) of a named general product."""
    if which == "rbf*matern52 d=2":
        o = gp.ProdKern([gp.Kern("rbf", np.array([0.6, 1.4]), 1.0, 0.0),
                         gp.Kern("matern52", 0.9, 1.0, 0.0)], 1.3, 0.05)
        k = mf.Kernel("rbf", [0.6, 1.4], 1.3, 0.05) * mf.Kernel("matern52", 0.9)
        return o, k, 2
    if which == "matern12*linear d=2":
        o = gp.ProdKern([gp.Kern("matern12", np.array([0.8, 1.2]), 1.0, 0.0),
                         gp.Kern("linear", 1.0, 1.0, 0.0)], 0.7, 0.1)
        k = mf.Kernel("matern12", [0.8, 1.2], 0.7, 0.1) * mf.Kernel("linear", 1.0)
        return o, k, 2
    if which == "linear*periodic*matern32 d=1":
        o = gp.ProdKern([gp.Kern("linear", 1.0, 1.0, 0.0), gp.Kern("periodic", 0.9, 1.0, 0.0, period=0.4),
                         gp.Kern("matern32", [1.1], 1.0, 0.0)], 0.9, 0.05)
        k = mf.Kernel("linear", 1.0, 0.9, 0.05) * mf.Kernel("periodic", 0.9, period=0.4) * mf.Kernel("matern32", [1.1])
        return o, k, 1
    if which == "matern32*matern52 d=3":
        o = gp.ProdKern([gp.Kern("matern32", np.array([0.7, 1.5, 1.1]), 1.0, 0.0),
                         gp.Kern("matern52", 1.3, 1.0, 0.0)], 1.1, 0.05)
        k = mf.Kernel("matern32", [0.7, 1.5, 1.1], 1.1, 0.05) * mf.Kernel("matern52", 1.3)
        return o, k, 3
    if which == "rbf*periodic*matern52*linear d=1":
        o = gp.ProdKern([gp.Kern("rbf", 1.7, 1.0, 0.0), gp.Kern("periodic", [0.8], 1.0, 0.0, period=0.35),
                         gp.Kern("matern52", 1.2, 1.0, 0.0), gp.Kern("linear", 1.0, 1.0, 0.0)], 0.8, 0.05)
        k = (mf.Kernel("rbf", 1.7, 0.8, 0.05) * mf.Kernel("periodic", [0.8], period=0.35)
             * mf.Kernel("matern52", 1.2) * mf.Kernel("linear", 1.0))
        return o, k, 1
    raise ValueError(which)


GENERAL = ["rbf*matern52 d=2", "matern12*linear d=2", "linear*periodic*matern32 d=1", "matern32*matern52 d=3",
           "rbf*periodic*matern52*linear d=1"]


@pytest.mark.parametrize("which", GENERAL)
@pytest.mark.parametrize("t", [1, 5, 33])
def test_general_product_matvec_vs_oracle(mf, which, t):
    banner(f"general product matvec {which} n=1237 t={t}")
    o, k, d = general(mf, which)
    X, _ = data(1300 + t, 1237, d)
    V = np.random.default_rng(1301 + t).standard_normal((1237, t)).astype(np.float32)
    ref = gp.ky_matvec(o, X.astype(np.float64), V.astype(np.float64))
    for precision in ("fp32", "fp32_valu", "fp32_direct", "fp32_gram"):
        out = host(mf.kernel_matvec(k, dev(X), dev(V), precision=precision))
        err = col_rel_err(out, ref).max()
        assert err <= 1e-5, (precision, err)
    # symmetric operator: u^T (K v) = v^T (K u)
    u = np.random.default_rng(1302).standard_normal((1237, 1)).astype(np.float32)
    ku = host(mf.kernel_matvec(k, dev(X), dev(u))).astype(np.float64)
    kv = host(mf.kernel_matvec(k, dev(X), dev(V[:, :1].copy()))).astype(np.float64)
    scale = float(np.abs(u[:, 0]) @ np.abs(ref[:, 0]))
    assert abs(float(u[:, 0] @ kv[:, 0]) - float(V[:, 0] @ ku[:, 0])) <= 1e-6 * scale


def test_general_product_rejects_bf16(mf):
    banner("general product: the bf16 forms are not offered")
    o, k, d = general(mf, "rbf*matern52 d=2")
    X, _ = data(1310, 300, d)
    V = np.ones((300, 3), np.float32)
    for form in ("bf16x1", "bf16x2", "bf16x3"):
        with pytest.raises(mf.MfgpError) as ei:
            mf.kernel_matvec(k, dev(X), dev(V), precision=form)
        assert ei.value.status == mf.UNSUPPORTED


@pytest.mark.parametrize("which", GENERAL)
def test_general_product_adjoint_vs_oracle(mf, which):
    banner(f"general product adjoint {which} n=900 t=3")
    o, k, d = general(mf, which)
    X, _ = data(1320, 900, d)
    rng = np.random.default_rng(1321)
    A = rng.standard_normal((900, 3)).astype(np.float32)
    B = rng.standard_normal((900, 3)).astype(np.float32)
    colw = [0.5, -0.25, 1.5]
    g = np.array(mf.kernel_adjoint(k, dev(X), dev(A), dev(B), colw))
    ref = gp.adjoint_bilinear(o, X, A, B, colw)
    assert len(g) == o.n_params(d) == k.n_params(d)
    print("adjoint", g, ref)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-4
    assert np.all(np.abs(g - ref) <= 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))


@pytest.mark.parametrize("which", ["rbf*matern52 d=2", "matern12*linear d=2", "rbf*periodic*matern52*linear d=1",
                                   "sum: matern32*linear + rbf"])
def test_general_product_mll_exact_mode_vs_cholesky_and_fd(mf, which):
    banner(f"general product exact-mode mll+grad {which} n=180")
    n = 180
    if which.startswith("sum"):
        d = 2
        o = gp.SumKern([gp.ProdKern([gp.Kern("matern32", 0.9, 1.0, 0.0), gp.Kern("linear", 1.0, 1.0, 0.0)], 0.6, 0.0),
                        gp.Kern("rbf", np.array([0.5, 1.1]), 0.8, 0.0)], 0.05)
        k = (mf.Kernel("matern32", 0.9, 0.6, 0.05) * mf.Kernel("linear", 1.0)) + mf.Kernel("rbf", [0.5, 1.1], 0.8)
    else:
        o, k, d = general(mf, which)
    X, y = data(1330, n, d)
    Z = (math.sqrt(n) * np.eye(n)).astype(np.float32)
    r = mf.mll_and_grad(k, dev(X), dev(y), Z=dev(Z), tol=1e-7)
    assert r["status"] == mf.OK, r["info"]
    Xd, yd = X.astype(np.float64), y.astype(np.float64)
    assert r["logdet"] == pytest.approx(gp.logdet(o, Xd), rel=1e-4)
    assert r["mll"] == pytest.approx(gp.mll(o, Xd, yd), rel=1e-4)
    ok_, rel = grad_ok(r["grad"], gp.mll_grad(o, Xd, yd))
    assert ok_, (r["grad"], rel)
    th = o.params(d)
    fd = []
    for q in range(len(th)):
        h = 1e-5 * th[q]
        tp, tm = th.copy(), th.copy()
        tp[q] += h
        tm[q] -= h
        fd.append((gp.mll(o.with_params(tp), Xd, yd) - gp.mll(o.with_params(tm), Xd, yd)) / (2 * h))
    ok_, rel = grad_ok(r["grad"], fd)
    assert ok_, (r["grad"], fd, rel)


@pytest.mark.parametrize("which", ["rbf*matern52 d=2", "matern12*linear d=2"])
def test_general_product_cg_predict_variance(mf, which):
    banner(f"general product {which}: CG, predictive mean and exact-mode variance n=1100 m=40")
    o, k, d = general(mf, which)
    X, y = data(1340, 1100, d)
    x, info, _, st = mf.cg_solve(k, dev(X), dev(y), tol=1e-6)
    assert st == mf.OK, info
    Xd = X.astype(np.float64)
    alpha = gp.solve(o, Xd, y.astype(np.float64))
    assert np.linalg.norm(host(x) - alpha) / np.linalg.norm(alpha) <= 1e-4
    Xs = np.random.default_rng(1341).uniform(-1.5, 2.5, (40, d)).astype(np.float32)
    mu = host(mf.predict_mean(k, dev(X), dev(Xs), x.float()))
    ref = gp.predict_mean(o, Xd, Xs.astype(np.float64), alpha)
    assert np.linalg.norm(mu - ref) / np.linalg.norm(ref) <= 1e-4
    # identity probes over the 40 test points: the exact latent variance,
    # whose prior k(x*, x*) carries the Linear factor's |x*|^2
    Z = (math.sqrt(40) * np.eye(40)).astype(np.float32)
    var, _, st = mf.predict_variance(k, dev(X), dev(Xs), Z=dev(Z), tol=1e-7)
    assert st == mf.OK
    vref = variance.predictive_variance(o, Xd, Xs)
    prior = variance.prior_variance(o, Xs)
    assert np.abs(host(var).astype(np.float64) - vref).max() <= 1e-4 * prior.max()


def test_general_product_rejected_by_the_preconditioner(mf):
    banner("general product: pivoted Cholesky is not offered")
    o, k, d = general(mf, "rbf*matern52 d=2")
    X, _ = data(1350, 200, d)
    with pytest.raises(mf.MfgpError) as ei:
        mf.pivoted_cholesky(k, dev(X), 8)
    assert ei.value.status == mf.UNSUPPORTED
