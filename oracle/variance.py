"""FP64 oracle: predictive variance, exact and by the stochastic diagonal estimator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

LightGP Sec. 2 ("Background") gives the posterior covariance at test points
X_* as Sigma_* = K_** - K_*f K_y^{-1} K_f*; its accuracy section reports that
the CG path estimates the variance with Rademacher probes (a Hutchinson-type
estimator), agreeing with the exact value to 3e-3.  Readings taken:

* The variance reported is the latent one, the diagonal of Sigma_*:
  v_m = k(x*_m, x*_m) - k_*m^T K_y^{-1} k_*m  (= s^2 - ... for every family
  here); the noise sigma^2 of a new observation is not added.
* The CG-path estimator is the stochastic diagonal estimator of Bekas,
  Kokiopoulou and Saad (2007) applied to A = K_*f K_y^{-1} K_f* (M x M): with
  probe columns z_c (M-vectors),
      diag(A)_m ~ sum_c z_mc (A z_c)_m / sum_c z_mc^2,
  and v_m = s^2 - diag(A)_m.  For Rademacher probes the denominator is p and
  the estimate is unbiased; for Z = the identity (p = M) it is exact.
* A z_c is formed as K_*f (K_y^{-1} (K_f* z_c)): two products with the
  rectangular kernel matrix and one solve with K_y.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve, solve_triangular

from . import gp


def prior_variance(kern: gp.Kern, Xs: np.ndarray) -> np.ndarray:
    """k(x, x) at every test point (s^2 for the stationary families here)."""
    Xs = np.asarray(Xs, dtype=np.float64)
    return np.array([gp.kernel_matrix(kern, Xs[m:m + 1], Xs[m:m + 1])[0, 0] for m in range(len(Xs))])


def predictive_variance(kern: gp.Kern, X: np.ndarray, Xs: np.ndarray) -> np.ndarray:
    """Exact latent variance: k(x*, x*) - |L^{-1} k_*|^2 with K_y = L L^T (Sec. 2)."""
    X = np.asarray(X, dtype=np.float64)
    Xs = np.asarray(Xs, dtype=np.float64)
    L = np.linalg.cholesky(gp.ky_matrix(kern, X))
    W = solve_triangular(L, gp.kernel_matrix(kern, X, Xs), lower=True)
    return prior_variance(kern, Xs) - np.sum(W * W, axis=0)


def probe_products(kern: gp.Kern, X: np.ndarray, Xs: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """A Z = K_*f K_y^{-1} K_f* Z with an exact (Cholesky) solve."""
    X = np.asarray(X, dtype=np.float64)
    Xs = np.asarray(Xs, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64).reshape(len(Xs), -1)
    Kfs = gp.kernel_matrix(kern, X, Xs)
    U = cho_solve(cho_factor(gp.ky_matrix(kern, X), lower=True), Kfs @ Z)
    return Kfs.T @ U


def diag_estimate(Z: np.ndarray, AZ: np.ndarray) -> np.ndarray:
    """sum_c z_mc (A z_c)_m / sum_c z_mc^2 (rows with an all-zero probe row give 0)."""
    Z = np.asarray(Z, dtype=np.float64)
    AZ = np.asarray(AZ, dtype=np.float64)
    num = np.sum(Z * AZ, axis=1)
    den = np.sum(Z * Z, axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def same_probe_variance(kern: gp.Kern, X: np.ndarray, Xs: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """The estimator with the given probes, every solve exact."""
    return prior_variance(kern, Xs) - diag_estimate(Z, probe_products(kern, X, Xs, Z))
