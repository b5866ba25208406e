"""Pins of the FP64 predictive-variance oracle (oracle/variance.py) to closed
forms, an independent computational route and the estimator's exact mode and
unbiasedness.  CPU only."""

import numpy as np
import pytest

from oracle import gp, variance
from paper_2605_17898_amd import inputs


def _kern(family="rbf", ls=0.4, s2=1.3, noise=0.05):
    return gp.Kern(family, ls, s2, noise)


@pytest.mark.parametrize("family", ["rbf", "matern12", "matern52"])
def test_variance_equals_joint_precision_route(family):
    # Sigma_* = ((J^{-1})_{**})^{-1} for the joint covariance J of (y, f_*):
    # the block-inverse (Schur complement) identity, a different computation
    # from the Cholesky solve of the oracle.
    rng = np.random.default_rng(1)
    X = rng.uniform(0, 1, (40, 2))
    Xs = rng.uniform(0, 1, (7, 2))
    k = _kern(family)
    Kfs = gp.kernel_matrix(k, X, Xs)
    J = np.block([[gp.ky_matrix(k, X), Kfs], [Kfs.T, gp.kernel_matrix(k, Xs, Xs)]])
    P = np.linalg.inv(J)[40:, 40:]
    ref = np.diag(np.linalg.inv(P))
    np.testing.assert_allclose(variance.predictive_variance(k, X, Xs), ref, rtol=1e-8, atol=1e-12)


def test_variance_single_training_point():
    # n = 1, x_* = x_1: v = s^2 - s^4 / (s^2 + sigma^2) = s^2 sigma^2 / (s^2 + sigma^2)
    k = _kern(s2=1.7, noise=0.2)
    X = np.array([[0.3, 0.6]])
    v = variance.predictive_variance(k, X, X)
    assert v[0] == pytest.approx(1.7 * 0.2 / 1.9, rel=1e-13)


def test_variance_far_test_point_is_prior():
    # every k(x_*, x_j) underflows to 0: v = s^2 exactly (no noise term)
    k = _kern(ls=0.1, s2=2.5)
    X = np.random.default_rng(2).uniform(0, 1, (30, 3))
    Xs = np.array([[50.0, 50.0, 50.0]])
    assert variance.predictive_variance(k, X, Xs)[0] == 2.5


def test_variance_far_apart_training_points():
    # K_y = (s^2 + sigma^2) I: v = s^2 - sum_j k(x_*, x_j)^2 / (s^2 + sigma^2)
    k = _kern(ls=0.05, s2=1.1, noise=0.3)
    X = np.array([[0.0, 0.0], [10.0, 0.0], [0.0, 10.0]])
    Xs = np.array([[0.02, -0.01], [10.03, 0.04]])
    kx = gp.kernel_matrix(k, X, Xs)
    ref = 1.1 - np.sum(kx ** 2, axis=0) / 1.4
    np.testing.assert_allclose(variance.predictive_variance(k, X, Xs), ref, rtol=1e-12)


def test_variance_bounds_and_monotone_in_data():
    # 0 < v <= s^2, and conditioning on one more point never raises v
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (25, 2))
    Xs = rng.uniform(0, 1, (12, 2))
    k = _kern()
    v = variance.predictive_variance(k, X, Xs)
    assert np.all(v > 0) and np.all(v <= 1.3)
    v2 = variance.predictive_variance(k, np.vstack([X, rng.uniform(0, 1, (1, 2))]), Xs)
    assert np.all(v2 <= v + 1e-12)


def test_estimator_exact_with_identity_probes():
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 1, (50, 3))
    Xs = rng.uniform(0, 1, (9, 3))
    k = _kern("matern32")
    got = variance.same_probe_variance(k, X, Xs, np.eye(9))
    np.testing.assert_allclose(got, variance.predictive_variance(k, X, Xs), rtol=1e-10, atol=1e-13)


def test_estimator_unbiased_over_probe_draws():
    # mean over 400 independent Rademacher draws of p = 4 probes is within
    # 4.5 standard errors of the exact variance at every test point
    rng = np.random.default_rng(5)
    X = rng.uniform(0, 1, (60, 2))
    Xs = rng.uniform(0, 1, (10, 2))
    k = _kern()
    exact = variance.predictive_variance(k, X, Xs)
    est = np.array([variance.same_probe_variance(k, X, Xs,
                                                 inputs.rademacher(np.random.default_rng(700 + s), 10, 4))
                    for s in range(400)])
    se = est.std(axis=0, ddof=1) / np.sqrt(len(est))
    assert np.all(np.abs(est.mean(axis=0) - exact) <= 4.5 * se + 1e-12)


def test_diag_estimate_handles_zero_probe_rows():
    Z = np.array([[1.0, -1.0], [0.0, 0.0]])
    AZ = np.array([[2.0, -4.0], [5.0, 6.0]])
    np.testing.assert_array_equal(variance.diag_estimate(Z, AZ), [3.0, 0.0])
