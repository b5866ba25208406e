"""Pins of the preconditioned-solver oracle (oracle/precond.py) against
definitions it does not use itself: full-rank factorisation, dense solves and
determinants, plain CG, Lanczos on the explicitly preconditioned matrix, and
exact-mode probes that make the stochastic estimators exact."""

import numpy as np
import pytest
from scipy.linalg import cholesky as dense_chol

from oracle import gp, krylov, precond
from oracle import brute


def _problem(n=60, d=2, seed=0, family="rbf", noise=0.05):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (n, d))
    y = np.sin(3 * X).sum(axis=1) + 0.1 * rng.standard_normal(n)
    return gp.Kern(family, [0.4] * d, 1.3, noise), X, y


@pytest.mark.parametrize("family", ["rbf", "matern12", "matern32", "matern52"])
def test_full_rank_pivoted_cholesky_reproduces_K(family):
    k, X, _ = _problem(40, 3, 1, family)
    L, piv = precond.pivoted_cholesky(k, X, 40)
    K = gp.kernel_matrix(gp.Kern(family, k.lengthscale, k.outputscale, 0.0), X, X)
    assert L.shape[1] == 40 and sorted(piv.tolist()) == list(range(40))
    np.testing.assert_allclose(L @ L.T, K, atol=1e-10 * np.abs(K).max())
    # permuted lower-triangular: row piv[m] vanishes after column m (to rounding)
    for m, i in enumerate(piv):
        assert np.all(np.abs(L[i, m + 1:]) <= 1e-8)
    # and it equals the dense Cholesky of the pivoted matrix
    C = dense_chol(K[np.ix_(piv, piv)], lower=True)
    np.testing.assert_allclose(L[piv], C, atol=1e-8)


def test_low_rank_error_and_greedy_pivots():
    k, X, _ = _problem(50, 2, 2)
    K = gp.kernel_matrix(gp.Kern("rbf", k.lengthscale, k.outputscale, 0.0), X, X)
    L, piv = precond.pivoted_cholesky(k, X, 7)
    E = K - L @ L.T
    assert np.linalg.eigvalsh(E).min() >= -1e-10          # Schur complement is PSD
    np.testing.assert_allclose(E[piv][:, piv], 0.0, atol=1e-10)
    # greedy: first pivot is index 0 (all diagonals equal s^2, ties to the smallest
    # index); each next pivot has the largest Schur-complement diagonal
    assert piv[0] == 0
    for m in range(1, 7):
        Lm = L[:, :m]
        dres = np.diag(K) - np.sum(Lm * Lm, axis=1)
        dres[piv[:m]] = -np.inf
        assert piv[m] == int(np.argmax(dres))
    # brute-force first column
    col = np.array([brute.entry("rbf", X[i], X[0], k.ls_vec(2), 1.3) for i in range(50)])
    np.testing.assert_allclose(L[:, 0], col / np.sqrt(1.3), rtol=1e-12)


def test_woodbury_solve_and_logdet_match_dense():
    k, X, _ = _problem(45, 2, 3)
    L, _ = precond.pivoted_cholesky(k, X, 9)
    P = L @ L.T + k.noise * np.eye(45)
    V = np.random.default_rng(1).standard_normal((45, 3))
    np.testing.assert_allclose(precond.precond_solve(L, k.noise, V), np.linalg.solve(P, V), rtol=1e-9)
    assert precond.precond_logdet(L, k.noise, 45) == pytest.approx(np.linalg.slogdet(P)[1], rel=1e-12)
    E = np.random.default_rng(2).standard_normal((9, 4))
    G = np.random.default_rng(3).standard_normal((45, 4))
    np.testing.assert_allclose(precond.precond_probes(L, k.noise, E, G), L @ E + np.sqrt(k.noise) * G)


def test_pcg_solves_and_reduces_to_plain_cg_without_factor():
    k, X, y = _problem(70, 2, 4)
    A = gp.ky_matrix(k, X)
    mm = lambda V: A @ V
    L, _ = precond.pivoted_cholesky(k, X, 10)
    B = np.stack([y, np.random.default_rng(5).standard_normal(70)], axis=1)
    Xs, al, be, it, bPb = precond.pcg(mm, L, k.noise, B, tol=1e-12)
    np.testing.assert_allclose(Xs, np.linalg.solve(A, B), rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(bPb, np.sum(B * precond.precond_solve(L, k.noise, B), axis=0))
    # k = 0: P = sigma^2 I, the iterates are plain CG's and T scales by 1/sigma^2
    L0 = np.zeros((70, 0))
    _, al0, be0, it0, _ = precond.pcg(mm, L0, k.noise, B[:, :1], tol=1e-12, max_iter=6)
    _, alc, bec, _ = krylov.cg(mm, B[:, :1], tol=1e-12, max_iter=6)
    d0, o0 = krylov.cg_to_tridiag(al0[0], be0[0])
    dc, oc = krylov.cg_to_tridiag(alc[0], bec[0])
    np.testing.assert_allclose(d0, dc / k.noise, rtol=1e-10)
    np.testing.assert_allclose(o0, oc / k.noise, rtol=1e-10)
    # fewer iterations than plain CG at the same tolerance
    _, _, _, itc = krylov.cg(mm, B, tol=1e-10)
    _, _, _, itp, _ = precond.pcg(mm, L, k.noise, B, tol=1e-10)
    assert np.all(itp < itc)


def test_pcg_tridiagonal_is_lanczos_of_split_preconditioned_matrix():
    k, X, y = _problem(60, 2, 6)
    A = gp.ky_matrix(k, X)
    L, _ = precond.pivoted_cholesky(k, X, 8)
    P = L @ L.T + k.noise * np.eye(60)
    w, Q = np.linalg.eigh(P)
    Pm = (Q / np.sqrt(w)) @ Q.T
    M = Pm @ A @ Pm
    _, al, be, _, _ = precond.pcg(lambda V: A @ V, L, k.noise, y[:, None], tol=1e-14, max_iter=6)
    d1, o1 = krylov.cg_to_tridiag(al[0][:6], be[0][:6])
    d2, o2 = krylov.lanczos(lambda v: M @ v, Pm @ y, 6)
    np.testing.assert_allclose(d1, d2, rtol=1e-8)
    np.testing.assert_allclose(np.abs(o1), np.abs(o2), rtol=1e-8)


def test_exact_mode_logdet_and_gradient():
    # w_c = sqrt(n) e_c, i.e. z_c = sqrt(n) P^{1/2} e_c: the estimators are exact.
    k, X, y = _problem(30, 2, 7)
    n = 30
    L, _ = precond.pivoted_cholesky(k, X, 5)
    P = L @ L.T + k.noise * np.eye(n)
    w, Q = np.linalg.eigh(P)
    Z = np.sqrt(n) * ((Q * np.sqrt(w)) @ Q.T)
    ld = precond.same_probe_logdet(k, X, L, Z)
    assert ld == pytest.approx(gp.logdet(k, X), rel=1e-10)
    g = precond.same_probe_grad(k, X, y, Z, L)
    np.testing.assert_allclose(g, gp.mll_grad(k, X, y), rtol=1e-8, atol=1e-10)


def test_pcg_slq_converged_equals_same_probe_logdet():
    k, X, _ = _problem(50, 2, 8)
    A = gp.ky_matrix(k, X)
    L, _ = precond.pivoted_cholesky(k, X, 6)
    rng = np.random.default_rng(9)
    Z = precond.precond_probes(L, k.noise, rng.standard_normal((6, 5)), rng.standard_normal((50, 5)))
    _, al, be, it, zPz = precond.pcg(lambda V: A @ V, L, k.noise, Z, tol=1e-13)
    q = [krylov.quadrature(*krylov.cg_to_tridiag(al[c], be[c]), zPz[c]) for c in range(5)]
    est = precond.precond_logdet(L, k.noise, 50) + float(np.mean(q))
    assert est == pytest.approx(precond.same_probe_logdet(k, X, L, Z), rel=1e-8)
