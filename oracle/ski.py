"""FP64 oracle of structured kernel interpolation (SKI / KISS-GP).

TEST INFRASTRUCTURE ONLY (see the package docstring).

LightGP Sec. 2 ("Structured kernel interpolation") and Sec. 3 ("Inference":
SKI with FFT) name the method of Wilson & Nickisch (2015) without its
details.  The reading taken here is that paper's: inducing points U on a
regular grid, K_XX ~ W K_UU W^T with W the local cubic convolution
interpolation of Keys (1981, a = -1/2; 4 grid nodes per dimension, 4^D
weights per row), so that

    K_y V ~ W K_UU W^T V + sigma^2 V,    mu_* ~ W_* K_UU W^T alpha.

Grid: per dimension k, m_k points with spacing h_k = r_k / (m_k - 4) and
first point lo_k = min_k - h_k, where min_k, max_k span the given point
sets and r_k = max_k - min_k (r_k = 1 when every point has the same
coordinate).  The last point is max_k + 2 h_k, so every point's stencil
(nodes b - 1 .. b + 2 of its cell b) lies on the grid.  Grid nodes are
flattened with dimension 0 fastest.  Everything is formed densely.
"""

from __future__ import annotations

import numpy as np

from . import gp


def grid(point_sets, m):
    """(lo [D], h [D]) of the grid covering every point set (see the module docstring)."""
    P = np.concatenate([np.asarray(p, dtype=np.float64).reshape(len(p), -1) for p in point_sets])
    mn, mx = P.min(axis=0), P.max(axis=0)
    r = mx - mn
    r = np.where(r > 0, r, 1.0)
    m = np.asarray(m, dtype=np.float64)
    h = r / (m - 4.0)
    return mn - h, h


def keys_weight(s: np.ndarray, a: float = -0.5) -> np.ndarray:
    """Keys' cubic convolution kernel u(s) (Keys 1981, with a = -1/2)."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    out = np.zeros_like(s)
    inner = s <= 1.0
    outer = (s > 1.0) & (s < 2.0)
    out[inner] = (a + 2.0) * s[inner] ** 3 - (a + 3.0) * s[inner] ** 2 + 1.0
    so = s[outer]
    out[outer] = a * so ** 3 - 5.0 * a * so ** 2 + 8.0 * a * so - 4.0 * a
    return out


def grid_points(lo, h, m) -> np.ndarray:
    """All grid nodes [prod m, D], dimension 0 fastest."""
    axes = [lo[k] + h[k] * np.arange(m[k]) for k in range(len(m))]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")           # last dimension slowest
    return np.stack([g.reshape(-1) for g in mesh[::-1]], axis=1)


def interp_matrix(X, lo, h, m) -> np.ndarray:
    """Dense W [N, prod m]: row i holds point i's 4^D cubic convolution weights."""
    X = np.asarray(X, dtype=np.float64).reshape(len(X), -1)
    n, d = X.shape
    M = int(np.prod(m))
    W = np.zeros((n, M))
    strides = np.cumprod([1] + list(m[:-1]))
    for i in range(n):
        per_dim = []
        for k in range(d):
            t = (X[i, k] - lo[k]) / h[k]
            b = int(np.floor(t))
            nodes = np.arange(b - 1, b + 3)
            per_dim.append((nodes, keys_weight(t - nodes)))
        for combo in np.ndindex(*([4] * d)):
            idx = 0
            w = 1.0
            for k in range(d):
                idx += per_dim[k][0][combo[k]] * strides[k]
                w *= per_dim[k][1][combo[k]]
            W[i, idx] += w
    return W


def ski_matrix(kern: gp.Kern, X1, X2, lo, h, m) -> np.ndarray:
    """W_1 K_UU W_2^T with K_UU = s^2 k(U, U) (no noise)."""
    U = grid_points(lo, h, m)
    return interp_matrix(X1, lo, h, m) @ gp.kernel_matrix(kern, U, U) @ interp_matrix(X2, lo, h, m).T


def ski_matvec(kern: gp.Kern, X, V, lo, h, m) -> np.ndarray:
    """(W K_UU W^T + sigma^2 I) V, the product the SKI solver iterates on."""
    V = np.asarray(V, dtype=np.float64)
    return ski_matrix(kern, X, X, lo, h, m) @ V + kern.noise * V


def ski_solve(kern: gp.Kern, X, B, lo, h, m) -> np.ndarray:
    A = ski_matrix(kern, X, X, lo, h, m)
    A[np.diag_indices_from(A)] += kern.noise
    return np.linalg.solve(A, np.asarray(B, dtype=np.float64))


# --------------------------------------------------------------------------
# Log marginal likelihood of the SKI model and its gradient (Sec. 2, the
# log p(y|X) formula, with K_ff replaced by W K_UU W^T on a fixed grid)
# --------------------------------------------------------------------------

def ski_ky(kern: gp.Kern, X, lo, h, m) -> np.ndarray:
    A = ski_matrix(kern, X, X, lo, h, m)
    A[np.diag_indices_from(A)] += kern.noise
    return A


def ski_mll(kern: gp.Kern, X, y, lo, h, m) -> float:
    """-1/2 [y^T A^{-1} y + log|A| + N log 2 pi], A = W K_UU W^T + sigma^2 I."""
    y = np.asarray(y, dtype=np.float64)
    L = np.linalg.cholesky(ski_ky(kern, X, lo, h, m))
    a = np.linalg.solve(L.T, np.linalg.solve(L, y))
    return -0.5 * (float(y @ a) + 2.0 * float(np.sum(np.log(np.diag(L)))) + len(y) * np.log(2.0 * np.pi))


def ski_dky(kern: gp.Kern, X, lo, h, m):
    """dA/dtheta in the kernel's gradient order: W (dK_UU/dtheta) W^T, then I."""
    W = interp_matrix(X, lo, h, m)
    U = grid_points(lo, h, m)
    mats = [W @ M @ W.T for M in gp.dky_matrices(kern, U)[:-1]]
    mats.append(np.eye(W.shape[0]))
    return mats


def ski_mll_grad(kern: gp.Kern, X, y, lo, h, m) -> np.ndarray:
    """Exact gradient: 1/2 a^T dA a - 1/2 tr(A^{-1} dA)."""
    A = ski_ky(kern, X, lo, h, m)
    a = np.linalg.solve(A, np.asarray(y, dtype=np.float64))
    Ainv = np.linalg.inv(A)
    return np.array([0.5 * float(a @ M @ a) - 0.5 * float(np.sum(Ainv * M)) for M in ski_dky(kern, X, lo, h, m)])


def ski_same_probe_grad(kern: gp.Kern, X, y, Z, lo, h, m) -> np.ndarray:
    """1/2 a^T dA a - 1/2 (1/p) sum_c u_c^T dA z_c with u_c = A^{-1} z_c (exact solves)."""
    A = ski_ky(kern, X, lo, h, m)
    Z = np.asarray(Z, dtype=np.float64)
    a = np.linalg.solve(A, np.asarray(y, dtype=np.float64))
    U = np.linalg.solve(A, Z)
    p = Z.shape[1]
    return np.array([0.5 * float(a @ M @ a) - 0.5 / p * float(np.sum(U * (M @ Z)))
                     for M in ski_dky(kern, X, lo, h, m)])
