"""FP64 oracle: pivoted-Cholesky preconditioner, preconditioned CG, SLQ and gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

LightGP Sec. 5 ("Limitations") names the comparison system's preconditioned,
batched CG as what its own plain CG loop lacks.  The preconditioned solver
checked here follows the published mBCG construction (Gardner et al. 2018,
GPyTorch) with the rank-k pivoted Cholesky factor of Harbrecht, Peters and
Schneider (2012).  Readings taken:

* Pivoted Cholesky of K = s^2 k(X, X) (the noise-free kernel matrix): the
  remaining diagonal starts at d = diag(K); at step m the pivot is
  i = argmax d (ties: the smallest index), the column is
  L[:, m] = (K[:, i] - L[:, :m] L[i, :m]^T) / sqrt(d_i), and d -= L[:, m]^2
  (d_i becomes exactly 0).  It stops early once max d <= 0.
* Preconditioner P = L L^T + s2n I (s2n = sigma^2).  P^{-1} v by the Woodbury
  identity: P^{-1} v = (v - L (s2n I_k + L^T L)^{-1} L^T v) / s2n, and
  log|P| = log|s2n I_k + L^T L| + (n - k) log s2n.
* Preconditioned CG from x0 = 0: z = P^{-1} r, alpha = r^T z / p^T A p,
  x += alpha p, r -= alpha A p, z' = P^{-1} r', beta = r'^T z' / r^T z,
  p = z' + beta p; a column stops when ||r|| / ||b|| <= tol (the unscaled
  residual, as in plain CG).
* Its (alpha, beta) give the Lanczos tridiagonal of P^{-1/2} A P^{-1/2} started
  at P^{-1/2} b, by the same map as plain CG (Saad Sec. 6.7.3 applied to the
  split-preconditioned system), and ||P^{-1/2} b||^2 = b^T P^{-1} b.
* Stochastic log-determinant: log|A| = log|P| + log|P^{-1/2} A P^{-1/2}|, the
  second term by SLQ with probes z_c ~ N(0, P), i.e. w_c = P^{-1/2} z_c ~
  N(0, I): q_c = (z_c^T P^{-1} z_c) e_1^T log(T_c) e_1.
* Gradient trace: tr(A^{-1} dA) ~ (1/p) sum_c (A^{-1} z_c)^T dA (P^{-1} z_c),
  unbiased for z ~ N(0, P) since E[P^{-1} z z^T] = I.
* Probes: z_c = L e_c + sqrt(s2n) g_c from standard normal draws e_c (k) and
  g_c (n), which are inputs (both sides receive the same draws).
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve, eigh

from . import gp, krylov


def pivoted_cholesky(kern: gp.Kern, X: np.ndarray, k: int):
    """Rank-k pivoted Cholesky of the noise-free K = s^2 k(X, X); returns (L [n, k'], pivots)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    k = min(k, n)
    if kern.family == "prod":
        noise_free = gp.ProdKern(kern.factors, kern.outputscale, 0.0)
    else:
        noise_free = gp.Kern(kern.family, kern.lengthscale, kern.outputscale, 0.0, period=kern.period)
    d = np.full(n, float(kern.outputscale))
    L = np.zeros((n, k))
    piv = []
    for m in range(k):
        i = int(np.argmax(d))
        if not d[i] > 0.0:
            return L[:, :m], np.array(piv, dtype=np.int64)
        col = gp.kernel_matrix(noise_free, X, X[i:i + 1])[:, 0]
        L[:, m] = (col - L[:, :m] @ L[i, :m]) / np.sqrt(d[i])
        d = d - L[:, m] ** 2
        d[i] = 0.0
        piv.append(i)
    return L, np.array(piv, dtype=np.int64)


def precond_solve(L: np.ndarray, s2n: float, V: np.ndarray) -> np.ndarray:
    """P^{-1} V with P = L L^T + s2n I, by the Woodbury identity."""
    V = np.asarray(V, dtype=np.float64)
    k = L.shape[1]
    if k == 0:
        return V / s2n
    S = s2n * np.eye(k) + L.T @ L
    return (V - L @ np.linalg.solve(S, L.T @ V)) / s2n


def precond_logdet(L: np.ndarray, s2n: float, n: int) -> float:
    k = L.shape[1]
    S = s2n * np.eye(k) + L.T @ L
    return float(np.linalg.slogdet(S)[1] + (n - k) * np.log(s2n)) if k else float(n * np.log(s2n))


def precond_probes(L: np.ndarray, s2n: float, E: np.ndarray, G: np.ndarray) -> np.ndarray:
    """z_c = L e_c + sqrt(s2n) g_c (columns of E [k, p] and G [n, p])."""
    return L @ np.asarray(E, dtype=np.float64) + np.sqrt(s2n) * np.asarray(G, dtype=np.float64)


def pcg(matmul, L: np.ndarray, s2n: float, B: np.ndarray, tol: float = 1e-10, max_iter=None):
    """Preconditioned CG on the columns of B; returns (X, alphas, betas, iters, b^T P^{-1} b)."""
    B = np.asarray(B, dtype=np.float64)
    B = B.reshape(B.shape[0], -1)
    n, t = B.shape
    max_iter = max_iter if max_iter is not None else min(n, 20000)
    X = np.zeros_like(B)
    R = B.copy()
    Zc = precond_solve(L, s2n, R)
    P = Zc.copy()
    rz = np.sum(R * Zc, axis=0)
    bPb = rz.copy()
    bnorm = np.linalg.norm(B, axis=0)
    active = bnorm > 0
    alphas = [[] for _ in range(t)]
    betas = [[] for _ in range(t)]
    iters = np.zeros(t, dtype=np.int64)
    for _ in range(max_iter):
        active &= np.linalg.norm(R, axis=0) > tol * bnorm
        if not active.any():
            break
        AP = matmul(P)
        for c in np.nonzero(active)[0]:
            a = rz[c] / float(P[:, c] @ AP[:, c])
            X[:, c] += a * P[:, c]
            R[:, c] -= a * AP[:, c]
            z = precond_solve(L, s2n, R[:, c])
            rz_new = float(R[:, c] @ z)
            b = rz_new / rz[c]
            P[:, c] = z + b * P[:, c]
            rz[c] = rz_new
            alphas[c].append(a)
            betas[c].append(b)
            iters[c] += 1
    return X, alphas, betas, iters, bPb


def _sym_pow(P: np.ndarray, power: float) -> np.ndarray:
    w, Q = eigh(P)
    return (Q * w ** power) @ Q.T


def same_probe_logdet(kern: gp.Kern, X: np.ndarray, L: np.ndarray, Z: np.ndarray) -> float:
    """log|P| + (1/p) sum_c w_c^T log(P^{-1/2} A P^{-1/2}) w_c, w_c = P^{-1/2} z_c, exactly."""
    A = gp.ky_matrix(kern, X)
    n = A.shape[0]
    P = L @ L.T + kern.noise * np.eye(n)
    Pm = _sym_pow(P, -0.5)
    W = Pm @ np.asarray(Z, dtype=np.float64).reshape(n, -1)
    return precond_logdet(L, kern.noise, n) + float(np.mean(krylov.quadform_log(Pm @ A @ Pm, W)))


def same_probe_grad(kern: gp.Kern, X: np.ndarray, y: np.ndarray, Z: np.ndarray,
                    L: np.ndarray) -> np.ndarray:
    """1/2 a^T dA a - 1/2 (1/p) sum_c (A^{-1} z_c)^T dA (P^{-1} z_c), every solve exact."""
    y = np.asarray(y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64).reshape(len(X), -1)
    p = Z.shape[1]
    c = cho_factor(gp.ky_matrix(kern, X), lower=True)
    a = cho_solve(c, y)
    U = cho_solve(c, Z)
    W = precond_solve(L, kern.noise, Z)
    return np.array([0.5 * float(a @ dA @ a) - 0.5 / p * float(np.sum(U * (dA @ W)))
                     for dA in gp.dky_matrices(kern, X)])
