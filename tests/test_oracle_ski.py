"""Pins of the SKI oracle (CPU only): the cubic convolution weights form a
partition of unity and reproduce linear and quadratic functions exactly
(Keys' kernel with a = -1/2 is exact for quadratics), data on grid nodes
make the SKI matrix the exact kernel matrix, the grid kernel matrix is
multilevel Toeplitz, and the SKI error against the exact kernel falls at the
cubic rate as the grid is refined."""

import numpy as np
import pytest

from oracle import gp, ski


@pytest.mark.parametrize("d", [1, 2, 3])
def test_weights_partition_of_unity_and_quadratic_exactness(d):
    rng = np.random.default_rng(d)
    X = rng.uniform(-1.0, 2.0, (40, d))
    m = [12, 9, 7][:d]
    lo, h = ski.grid([X], m)
    W = ski.interp_matrix(X, lo, h, m)
    U = ski.grid_points(lo, h, m)
    assert np.all(np.count_nonzero(W, axis=1) <= 4 ** d)
    np.testing.assert_allclose(W.sum(axis=1), 1.0, rtol=0, atol=1e-13)
    for k in range(d):
        np.testing.assert_allclose(W @ U[:, k], X[:, k], rtol=0, atol=1e-12)
        np.testing.assert_allclose(W @ U[:, k] ** 2, X[:, k] ** 2, rtol=0, atol=1e-11)
    # cubic terms are not reproduced (the stencil is third-order accurate only)
    assert np.abs(W @ U[:, 0] ** 3 - X[:, 0] ** 3).max() > 1e-6


def test_grid_covers_stencils():
    X = np.array([[0.0], [1.0], [0.37]])
    lo, h = ski.grid([X], [20])
    assert h[0] == pytest.approx(1.0 / 16)
    assert lo[0] == pytest.approx(-1.0 / 16)
    t = (X[:, 0] - lo[0]) / h[0]
    assert np.all(np.floor(t) - 1 >= 0) and np.all(np.floor(t) + 2 <= 19)


def test_on_grid_data_is_exact():
    lo, h, m = np.array([-0.5, 0.0]), np.array([0.25, 0.2]), [10, 8]
    U = ski.grid_points(lo, h, m)
    X = U[np.random.default_rng(0).choice(len(U), 25, replace=False)]
    # interior nodes only, so the stencil stays on the grid
    X = X[(X[:, 0] > lo[0] + h[0]) & (X[:, 0] < lo[0] + 7 * h[0]) & (X[:, 1] > lo[1] + h[1])
          & (X[:, 1] < lo[1] + 5 * h[1])]
    k = gp.Kern("matern32", np.array([0.4, 0.7]), 1.2, 0.0)
    np.testing.assert_allclose(ski.ski_matrix(k, X, X, lo, h, m), gp.kernel_matrix(k, X, X), rtol=0,
                               atol=1e-13)


def test_grid_kernel_is_multilevel_toeplitz():
    lo, h, m = np.array([0.0, 0.0]), np.array([0.1, 0.3]), [6, 5]
    U = ski.grid_points(lo, h, m)
    K = gp.kernel_matrix(gp.Kern("rbf", np.array([0.3, 0.8]), 1.0, 0.0), U, U)
    idx = np.stack(np.unravel_index(np.arange(30), (5, 6))[::-1], axis=1)   # (j0, j1) of each node
    for a in range(30):
        for b in range(30):
            off = np.abs(idx[a] - idx[b])
            assert K[a, b] == pytest.approx(K[0, off[0] + 6 * off[1]], rel=1e-14)


@pytest.mark.parametrize("family", ["rbf", "matern52"])
def test_ski_error_falls_cubically(family):
    rng = np.random.default_rng(5)
    X = rng.uniform(0.0, 1.0, (60, 1))
    k = gp.Kern(family, 0.3, 1.0, 0.0)
    K = gp.kernel_matrix(k, X, X)
    errs = []
    for m in (24, 48, 96):
        lo, h = ski.grid([X], [m])
        errs.append(np.abs(ski.ski_matrix(k, X, X, lo, h, [m]) - K).max())
    # h halves (about) at each step: an O(h^3) scheme gains about 8x
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5


@pytest.mark.parametrize("family,ard", [("rbf", True), ("matern32", False), ("matern52", True),
                                        ("matern12", False), ("periodic", True)])
def test_ski_mll_gradient_central_differences(family, ard):
    # the grid is fixed by the data, so the SKI MLL is a smooth function of theta
    rng = np.random.default_rng(11)
    X = rng.uniform(0.0, 1.0, (45, 2))
    y = np.sin(4 * X[:, 0]) + 0.1 * rng.standard_normal(45)
    ls = np.array([0.3, 0.5]) if ard else 0.4
    k = gp.Kern(family, ls, 1.1, 0.05, period=0.7)
    lo, h = ski.grid([X], [14, 12])
    g = ski.ski_mll_grad(k, X, y, lo, h, [14, 12])
    th = k.params(2)
    for q in range(len(th)):
        e = 1e-6 * th[q]
        tp, tm = th.copy(), th.copy()
        tp[q] += e
        tm[q] -= e
        fd = (ski.ski_mll(k.with_params(tp), X, y, lo, h, [14, 12])
              - ski.ski_mll(k.with_params(tm), X, y, lo, h, [14, 12])) / (2 * e)
        assert g[q] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(g).max())


def test_ski_same_probe_grad_exact_mode_is_exact():
    # probes sqrt(N) e_c make the Hutchinson trace exact
    rng = np.random.default_rng(12)
    X = rng.uniform(0.0, 1.0, (30, 1))
    y = rng.standard_normal(30)
    k = gp.Kern("rbf", 0.2, 1.0, 0.1)
    lo, h = ski.grid([X], [40])
    Z = np.sqrt(30) * np.eye(30)
    np.testing.assert_allclose(ski.ski_same_probe_grad(k, X, y, Z, lo, h, [40]),
                               ski.ski_mll_grad(k, X, y, lo, h, [40]), rtol=1e-9)
