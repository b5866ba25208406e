"""Pins of the oracle's Linear kernel and of kernel sums (CPU only).

Linear k = s^2 x.x' is Bayesian linear regression with weights w ~ N(0, s^2 I):
its log marginal likelihood and predictive mean are checked against the
weight-space forms (matrix determinant lemma, Woodbury, ridge regression),
which never form the N x N kernel.  Sums are checked against brute-force
entries, against scipy's multivariate normal log-density with that
covariance, against the identity RBF(l, a) + RBF(l, b) = RBF(l, a + b), and
by central differences of the exact MLL in every parameter."""

import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import brute, gp, variance


def _data(seed, n, d):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 2, (n, d))
    y = X @ rng.standard_normal(d) + np.sin(3 * X[:, 0]) + 0.1 * rng.standard_normal(n)
    return X, y


def test_linear_entries_brute_force():
    X, _ = _data(0, 10, 3)
    k = gp.Kern("linear", 1.0, 0.7, 0.1)
    K = gp.kernel_matrix(k, X, X)
    for i in range(10):
        for j in range(10):
            assert K[i, j] == pytest.approx(brute.entry("linear", X[i], X[j], None, 0.7), rel=1e-13, abs=1e-15)


def test_linear_mll_equals_weight_space_evidence():
    # y ~ N(0, sigma^2 I + s^2 X X^T):
    #   log|K_y| = n log sigma^2 + log|I_d + (s^2 / sigma^2) X^T X|
    #   y^T K_y^{-1} y = (y^T y - y^T X (sigma^2 / s^2 I + X^T X)^{-1} X^T y) / sigma^2
    X, y = _data(1, 60, 3)
    s2, sn = 0.8, 0.05
    k = gp.Kern("linear", 1.0, s2, sn)
    G = X.T @ X
    ld = 60 * math.log(sn) + np.linalg.slogdet(np.eye(3) + (s2 / sn) * G)[1]
    Xy = X.T @ y
    quad = (y @ y - Xy @ np.linalg.solve(sn / s2 * np.eye(3) + G, Xy)) / sn
    ref = -0.5 * (quad + ld + 60 * math.log(2 * math.pi))
    assert gp.mll(k, X, y) == pytest.approx(ref, rel=1e-11)
    assert gp.logdet(k, X) == pytest.approx(ld, rel=1e-11)


def test_linear_predictive_mean_is_ridge_regression():
    X, y = _data(2, 50, 2)
    Xs = np.random.default_rng(3).uniform(-2, 3, (17, 2))
    s2, sn = 1.3, 0.2
    k = gp.Kern("linear", 1.0, s2, sn)
    mu = gp.predict_mean(k, X, Xs, gp.solve(k, X, y))
    w = np.linalg.solve(X.T @ X + sn / s2 * np.eye(2), X.T @ y)
    np.testing.assert_allclose(mu, Xs @ w, rtol=1e-10, atol=1e-12)


def test_linear_rank_and_prior_variance():
    X, _ = _data(4, 30, 3)
    k = gp.Kern("linear", 1.0, 2.0, 0.1)
    ev = np.linalg.eigvalsh(gp.kernel_matrix(k, X, X))
    assert np.all(np.abs(ev[:-3]) <= 1e-10 * ev[-1])      # rank d
    np.testing.assert_allclose(variance.prior_variance(k, X), 2.0 * np.sum(X * X, axis=1), rtol=1e-13)


def _sum():
    return gp.SumKern([gp.Kern("rbf", np.array([0.4, 0.9]), 1.1, 0.0),
                       gp.Kern("periodic", 0.7, 0.6, 0.0, period=0.45),
                       gp.Kern("linear", 1.0, 0.3, 0.0)], 0.04)


def test_sum_entries_brute_force_and_mvn_logpdf():
    X, y = _data(5, 25, 2)
    k = _sum()
    K = gp.kernel_matrix(k, X, X)
    C = np.zeros((25, 25))
    for i in range(25):
        for j in range(25):
            C[i, j] = (brute.entry("rbf", X[i], X[j], [0.4, 0.9], 1.1)
                       + brute.entry("periodic", X[i], X[j], [0.7, 0.7], 0.6, period=0.45)
                       + brute.entry("linear", X[i], X[j], None, 0.3))
    np.testing.assert_allclose(K, C, rtol=1e-12, atol=1e-14)
    ref = multivariate_normal(mean=np.zeros(25), cov=C + 0.04 * np.eye(25)).logpdf(y)
    assert gp.mll(k, X, y) == pytest.approx(ref, rel=1e-10)


def test_sum_of_rbf_with_one_lengthscale_is_rbf():
    X, _ = _data(6, 20, 3)
    a = gp.SumKern([gp.Kern("rbf", 0.5, 0.7, 0.0), gp.Kern("rbf", 0.5, 1.9, 0.0)], 0.1)
    b = gp.Kern("rbf", 0.5, 2.6, 0.1)
    np.testing.assert_allclose(gp.ky_matrix(a, X), gp.ky_matrix(b, X), rtol=1e-13)


def test_sum_param_order_round_trip():
    k = _sum()
    th = k.params(2)
    # [l_1, l_2, s2_rbf, l_per, p, s2_per, s2_lin, sigma^2]
    np.testing.assert_array_equal(th, [0.4, 0.9, 1.1, 0.7, 0.45, 0.6, 0.3, 0.04])
    assert k.n_params(2) == 8
    np.testing.assert_array_equal(k.with_params(th).params(2), th)


@pytest.mark.parametrize("which", ["sum", "linear"])
def test_mll_gradient_central_differences(which):
    X, y = _data(7, 40, 2)
    k = _sum() if which == "sum" else gp.Kern("linear", 1.0, 0.5, 0.07)
    g = gp.mll_grad(k, X, y)
    th = k.params(2)
    assert len(g) == len(th)
    for q in range(len(th)):
        h = 1e-6 * th[q]
        tp, tm = th.copy(), th.copy()
        tp[q] += h
        tm[q] -= h
        fd = (gp.mll(k.with_params(tp), X, y) - gp.mll(k.with_params(tm), X, y)) / (2 * h)
        assert g[q] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(g).max())
