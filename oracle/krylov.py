"""FP64 oracle: conjugate gradients, Lanczos and the stochastic Lanczos log-determinant.

TEST INFRASTRUCTURE ONLY (see the package docstring).

LightGP Sec. 2 ("CG-based inference") replaces the Cholesky solve by conjugate
gradients that only need products K_y v; Sec. 3 ("Inference") pairs the CG
solver with a stochastic Lanczos log-determinant, and Sec. 5 says the CG loop
is plain: no preconditioner, no batching tricks.  The reading taken here:

* CG starts from x0 = 0, is unpreconditioned, and stops a column once
  ||r_c||_2 / ||b_c||_2 <= tol; a converged column freezes.  A zero right-hand
  side returns x = 0 after zero iterations.
* The Lanczos tridiagonal of a CG run started at x0 = 0 follows from its step
  sizes alpha_j and ratios beta_j = r_{j+1}^T r_{j+1} / r_j^T r_j
  (Saad, Iterative Methods for Sparse Linear Systems, Sec. 6.7.3):
      T_jj     = 1/alpha_j + beta_{j-1}/alpha_{j-1}   (second term absent at j = 0)
      T_j,j+1  = sqrt(beta_j) / alpha_j
* Stochastic Lanczos quadrature (Ubaru, Chen & Saad 2017): for a probe z,
  z^T log(A) z ~= ||z||^2 sum_k S_0k^2 log(theta_k) with T = S diag(theta) S^T;
  log|A| ~= (1/p) sum_c of that over the probes.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def cg(matmul, B: np.ndarray, tol: float = 1e-10, max_iter: int | None = None):
    """Plain FP64 CG on the columns of B, all columns stepped together.

    Returns (X, alphas, betas, iters) where alphas[c] / betas[c] are the lists
    of step sizes and residual-norm ratios of column c and iters[c] its count.
    """
    B = np.asarray(B, dtype=np.float64)
    squeeze = B.ndim == 1
    B = B.reshape(B.shape[0], -1)
    n, t = B.shape
    max_iter = max_iter if max_iter is not None else min(n, 20000)
    X = np.zeros_like(B)
    R = B.copy()
    P = R.copy()
    rr = np.sum(R * R, axis=0)
    bnorm = np.sqrt(rr.copy())
    active = bnorm > 0
    alphas = [[] for _ in range(t)]
    betas = [[] for _ in range(t)]
    iters = np.zeros(t, dtype=np.int64)
    for _ in range(max_iter):
        active &= np.sqrt(rr) > tol * bnorm
        if not active.any():
            break
        AP = matmul(P)
        pap = np.sum(P * AP, axis=0)
        for c in np.nonzero(active)[0]:
            a = rr[c] / pap[c]
            X[:, c] += a * P[:, c]
            R[:, c] -= a * AP[:, c]
            rr_new = float(R[:, c] @ R[:, c])
            b = rr_new / rr[c]
            P[:, c] = R[:, c] + b * P[:, c]
            rr[c] = rr_new
            alphas[c].append(a)
            betas[c].append(b)
            iters[c] += 1
    return (X[:, 0] if squeeze else X), alphas, betas, iters


def cg_to_tridiag(alphas, betas):
    """Lanczos tridiagonal (diag, offdiag) from CG coefficients (Saad Sec. 6.7.3)."""
    a = np.asarray(alphas, dtype=np.float64)
    b = np.asarray(betas, dtype=np.float64)
    m = len(a)
    diag = 1.0 / a
    diag[1:] += b[:m - 1] / a[:m - 1]
    off = np.sqrt(b[:m - 1]) / a[:m - 1]
    return diag, off


def lanczos(matmul, z: np.ndarray, m: int):
    """m steps of Lanczos from z/||z|| with full reorthogonalisation (FP64)."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    Q = np.zeros((n, m + 1))
    Q[:, 0] = z / np.linalg.norm(z)
    diag = np.zeros(m)
    off = np.zeros(max(m - 1, 0))
    for j in range(m):
        w = matmul(Q[:, j])
        diag[j] = Q[:, j] @ w
        w = w - Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        w = w - Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        if j < m - 1:
            off[j] = np.linalg.norm(w)
            Q[:, j + 1] = w / off[j]
    return diag, off


def quadrature(diag, off, znorm2: float) -> float:
    """||z||^2 e_1^T log(T) e_1 via the eigen-decomposition of the tridiagonal T."""
    theta, S = eigh_tridiagonal(np.asarray(diag, dtype=np.float64), np.asarray(off, dtype=np.float64))
    return float(znorm2 * np.sum(S[0, :] ** 2 * np.log(theta)))


def quadform_log(A: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Exact z_c^T log(A) z_c for every column via a dense symmetric eigen-solve."""
    w, Q = np.linalg.eigh(np.asarray(A, dtype=np.float64))
    P = Q.T @ np.asarray(Z, dtype=np.float64).reshape(A.shape[0], -1)
    return np.sum(P * P * np.log(w)[:, None], axis=0)


def slq_logdet(matmul, Z: np.ndarray, tol: float = 1e-10, max_iter: int | None = None):
    """Stochastic Lanczos log|A| from FP64 CG runs on the probe columns.

    Returns (estimate, per-probe quadratures, per-probe Lanczos lengths).
    """
    Z = np.asarray(Z, dtype=np.float64)
    _, al, be, it = cg(matmul, Z, tol=tol, max_iter=max_iter)
    q = np.array([quadrature(*cg_to_tridiag(al[c], be[c]), float(Z[:, c] @ Z[:, c]))
                  for c in range(Z.shape[1])])
    return float(np.mean(q)), q, it
