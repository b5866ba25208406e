"""Predictive variance on the CG path (stochastic diagonal estimator of
K_*f K_y^{-1} K_f*) against the FP64 oracle (oracle/variance.py).

The GPU result is compared with the oracle evaluating the same estimator with
the same probes and exact (Cholesky) solves, and, with identity probes, with
the exact variance.  The difference comes from the CG solve (stopped at a
relative residual of 1e-6 of each right-hand side K_f* z_c) and the FP32
entries; the bound used, 1e-4 s^2 absolute, is the CG-path analogue of the
1e-5 variance agreement reported for the exact paths.
"""

import numpy as np
import pytest

from oracle import probes as oprobes
from oracle import variance
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, dev, host, mkern, okern

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


def _setup(seed, n, m, d, family, noise=0.05):
    w = inputs.random_problem(seed, n, d, family, ard=True, noise=noise)
    Xs = np.random.default_rng(seed + 1).uniform(-0.1, 1.1, (m, d)).astype(np.float32)
    return w, Xs


@pytest.mark.parametrize("family", ["rbf", "matern12", "matern52"])
def test_variance_same_probe(mf, family):
    banner(f"predict_variance {family} n=1500 m=203 p=16 vs same-probe oracle")
    w, Xs = _setup(700, 1500, 203, 2, family)
    Z = inputs.rademacher(np.random.default_rng(701), 203, 16)
    var, info, st = mf.predict_variance(mkern(w), dev(w.X), dev(Xs), Z=dev(Z), tol=1e-6)
    assert st == mf.OK, info
    ref = variance.same_probe_variance(okern(w), w.X, Xs, Z)
    err = np.abs(host(var).astype(np.float64) - ref).max()
    print(f"max |var - same-probe oracle| = {err:.2e} (s2 = {w.outputscale})")
    assert err <= 1e-4 * w.outputscale


def test_variance_exact_mode(mf):
    # identity probes make the estimator exact: the exact predictive variance
    banner("predict_variance exact mode: Z = I_48, n=900 vs Cholesky variance")
    w, Xs = _setup(702, 900, 48, 3, "matern32")
    var, _, st = mf.predict_variance(mkern(w), dev(w.X), dev(Xs), Z=dev(np.eye(48, dtype=np.float32)), tol=1e-7)
    assert st == mf.OK
    ref = variance.predictive_variance(okern(w), w.X, Xs)
    err = np.abs(host(var).astype(np.float64) - ref).max()
    print(f"max |var - exact| = {err:.2e}")
    assert err <= 1e-4 * w.outputscale


def test_variance_seeded_probes(mf):
    # Z = NULL: SplitMix64 Rademacher probes over the test points, the same
    # stream as mfgp_rademacher (the oracle's own implementation of it here)
    banner("predict_variance seeded probes (seed 17, p=33) vs oracle on the same draws")
    w, Xs = _setup(703, 1200, 150, 4, "rbf")
    var, _, st = mf.predict_variance(mkern(w), dev(w.X), dev(Xs), num_probes=33, seed=17, tol=1e-6)
    assert st == mf.OK
    Z = oprobes.rademacher(17, 150, 33)
    ref = variance.same_probe_variance(okern(w), w.X, Xs, Z)
    assert np.abs(host(var).astype(np.float64) - ref).max() <= 1e-4 * w.outputscale


@pytest.mark.parametrize("n,m,p", [(1, 1, 1), (5, 3, 2), (257, 1, 7), (64, 300, 1)])
def test_variance_small_shapes(mf, n, m, p):
    banner(f"predict_variance shapes n={n} m={m} p={p}")
    w, Xs = _setup(704, n, m, 2, "rbf", noise=0.1)
    Z = inputs.rademacher(np.random.default_rng(705), m, p)
    var, _, st = mf.predict_variance(mkern(w), dev(w.X), dev(Xs), Z=dev(Z), tol=1e-7)
    assert st == mf.OK
    ref = variance.same_probe_variance(okern(w), w.X, Xs, Z)
    assert np.abs(host(var).astype(np.float64) - ref).max() <= 1e-4 * w.outputscale


def test_variance_far_test_points_are_prior(mf):
    # test points far from every training point: K_f* = 0, var = s^2 exactly
    banner("predict_variance far test points give s^2")
    w, _ = _setup(706, 500, 10, 2, "rbf")
    Xs = np.full((10, 2), 100.0, np.float32)
    Z = inputs.rademacher(np.random.default_rng(707), 10, 4)
    var, _, st = mf.predict_variance(mkern(w), dev(w.X), dev(Xs), Z=dev(Z))
    assert st == mf.OK
    np.testing.assert_array_equal(host(var), np.float32(w.outputscale))
