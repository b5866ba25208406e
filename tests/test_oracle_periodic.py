"""Pins of the oracle's periodic kernel (exp-sine-squared, ARD lengthscales,
one period): brute-force entries, periodicity, the half-period closed form,
the RBF-on-features identity and central differences of the exact MLL in
every parameter including the period.  CPU only."""

import math

import numpy as np
import pytest

from oracle import brute, gp


def _kern(ls=(0.7, 1.3), s2=1.4, noise=0.05, p=0.8):
    return gp.Kern("periodic", np.asarray(ls, dtype=np.float64), s2, noise, period=p)


def test_periodic_entries_brute_force():
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 2, (12, 2))
    k = _kern()
    K = gp.kernel_matrix(k, X, X)
    for i in range(12):
        for j in range(12):
            assert K[i, j] == pytest.approx(brute.entry("periodic", X[i], X[j], k.ls_vec(2), 1.4, period=0.8),
                                            rel=1e-13)


def test_periodic_shift_by_period_and_half_period():
    k = _kern(ls=(0.6, 0.9), p=1.7)
    x = np.array([[0.3, -0.4]])
    shifted = x + np.array([[1.7, 0.0]])
    assert gp.kernel_matrix(k, x, shifted)[0, 0] == pytest.approx(1.4, rel=1e-14)
    half = x + np.array([[0.0, 0.85]])   # sin^2 = 1 in dimension 2 only
    assert gp.kernel_matrix(k, x, half)[0, 0] == pytest.approx(1.4 * math.exp(-2.0 / 0.81), rel=1e-13)


def test_periodic_equals_rbf_on_circle_features():
    # sum_k 2 sin^2(pi D_k / p) / l_k^2 = 1/2 |phi_i - phi_j|^2 with
    # phi_k = (cos(2 pi x_k / p), sin(2 pi x_k / p)) / l_k
    rng = np.random.default_rng(1)
    X1 = rng.uniform(-3, 3, (9, 3))
    X2 = rng.uniform(-3, 3, (7, 3))
    ls, p = np.array([0.5, 1.1, 2.0]), 1.3
    k = gp.Kern("periodic", ls, 0.9, 0.1, period=p)

    def phi(X):
        a = 2 * np.pi * X / p
        return np.concatenate([np.cos(a) / ls, np.sin(a) / ls], axis=1)

    krbf = gp.Kern("rbf", 1.0, 0.9, 0.1)
    np.testing.assert_allclose(gp.kernel_matrix(k, X1, X2), gp.kernel_matrix(krbf, phi(X1), phi(X2)),
                               rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("ard", [True, False])
def test_periodic_mll_gradient_central_differences(ard):
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 2, (40, 2))
    y = np.sin(3 * X[:, 0]) + 0.1 * rng.standard_normal(40)
    k = _kern() if ard else gp.Kern("periodic", 0.9, 1.4, 0.05, period=0.8)
    g = gp.mll_grad(k, X, y)
    theta = k.params(2)
    assert len(g) == len(theta) == (5 if ard else 4)
    for q in range(len(theta)):
        h = 1e-5 * theta[q]
        tp, tm = theta.copy(), theta.copy()
        tp[q] += h
        tm[q] -= h
        fd = (gp.mll(k.with_params(tp), X, y) - gp.mll(k.with_params(tm), X, y)) / (2 * h)
        assert g[q] == pytest.approx(fd, rel=1e-5, abs=1e-6 * np.abs(g).max())
