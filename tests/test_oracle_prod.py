"""Pins of the oracle's kernel products (CPU only): brute-force entries, the
closed form RBF(l_a) * RBF(l_b) = RBF with 1/l^2 = 1/l_a^2 + 1/l_b^2, the
RBF * Periodic product as RBF on concatenated features, scipy's MVN
log-density, and central differences of the exact MLL in every parameter of
a product and of a sum that holds one."""

import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import brute, gp


def _X(seed, n, d):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 2, (n, d)), rng.standard_normal(n)


def _rbf_per(s2=1.3, noise=0.05):
    return gp.ProdKern([gp.Kern("rbf", np.array([0.6, 1.4]), 1.0, 0.0),
                        gp.Kern("periodic", 0.8, 1.0, 0.0, period=0.45)], s2, noise)


def test_product_brute_force_and_mvn():
    X, y = _X(0, 20, 2)
    k = _rbf_per()
    C = np.zeros((20, 20))
    for i in range(20):
        for j in range(20):
            C[i, j] = (brute.entry("rbf", X[i], X[j], [0.6, 1.4], 1.3)
                       * brute.entry("periodic", X[i], X[j], [0.8, 0.8], 1.0, period=0.45))
    np.testing.assert_allclose(gp.kernel_matrix(k, X, X), C, rtol=1e-12, atol=1e-15)
    ref = multivariate_normal(mean=np.zeros(20), cov=C + 0.05 * np.eye(20)).logpdf(y)
    assert gp.mll(k, X, y) == pytest.approx(ref, rel=1e-10)


def test_product_of_rbfs_is_rbf():
    X, _ = _X(1, 15, 3)
    la, lb = np.array([0.5, 0.9, 1.3]), 0.7
    k = gp.ProdKern([gp.Kern("rbf", la, 1.0, 0.0), gp.Kern("rbf", lb, 1.0, 0.0)], 0.8, 0.1)
    lc = 1.0 / np.sqrt(1.0 / la ** 2 + 1.0 / lb ** 2)
    np.testing.assert_allclose(gp.ky_matrix(k, X), gp.ky_matrix(gp.Kern("rbf", lc, 0.8, 0.1), X), rtol=1e-13)


def test_rbf_times_periodic_is_rbf_on_concatenated_features():
    X1, _ = _X(2, 9, 2)
    X2, _ = _X(3, 7, 2)
    lr, lp, p = np.array([0.6, 1.4]), 0.8, 0.45

    def phi(X):
        a = 2 * np.pi * X / p
        return np.concatenate([X / lr, np.cos(a) / lp, np.sin(a) / lp], axis=1)

    np.testing.assert_allclose(gp.kernel_matrix(_rbf_per(), X1, X2),
                               gp.kernel_matrix(gp.Kern("rbf", 1.0, 1.3, 0.0), phi(X1), phi(X2)),
                               rtol=1e-12, atol=1e-15)


def test_param_order():
    k = _rbf_per()
    # [l_r1, l_r2 | l_p, p | s2, sigma^2]
    np.testing.assert_array_equal(k.params(2), [0.6, 1.4, 0.8, 0.45, 1.3, 0.05])
    np.testing.assert_array_equal(k.with_params(k.params(2)).params(2), k.params(2))
    ks = gp.SumKern([k, gp.Kern("linear", 1.0, 0.3, 0.0)], 0.05)
    np.testing.assert_array_equal(ks.params(2), [0.6, 1.4, 0.8, 0.45, 1.3, 0.3, 0.05])


@pytest.mark.parametrize("which", ["prod", "sum_with_prod"])
def test_mll_gradient_central_differences(which):
    X, y = _X(4, 40, 2)
    k = _rbf_per()
    if which == "sum_with_prod":
        k = gp.SumKern([k, gp.Kern("matern32", 0.5, 0.4, 0.0)], 0.05)
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
