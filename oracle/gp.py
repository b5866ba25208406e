"""FP64 oracle: kernel entries, K_y products, exact GP solve, mean, MLL, gradients.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Everything here is the
plain definition, formed densely in float64 with numpy/scipy.

Kernel parametrisation.  LightGP Sec. 3 ("Kernels") names the families RBF and
Matern-1/2, 3/2, 5/2 and a ``Scale`` wrapper but prints no formulas.  The
reading taken here is the standard one (Rasmussen & Williams, ch. 4), with the
1/2 inside the RBF exponent, a lengthscale per input dimension (ARD) or one
shared lengthscale, an outputscale s^2 (the ``Scale`` variance) and a noise
variance sigma^2 (Sec. 2, the sigma_n^2 of K_y = K_ff + sigma_n^2 I):

    r^2 = sum_k ((x_k - x'_k) / l_k)^2,   rho = sqrt(r^2)
    RBF        k = s^2 exp(-r^2 / 2)
    Matern-1/2 k = s^2 exp(-rho)
    Matern-3/2 k = s^2 (1 + sqrt3 rho) exp(-sqrt3 rho)
    Matern-5/2 k = s^2 (1 + sqrt5 rho + 5 rho^2 / 3) exp(-sqrt5 rho)

Distances are formed by direct differences, never by the ||x||^2 + ||x'||^2 -
2 x.x' expansion.

Gradient order everywhere: [l_1 .. l_d] (ARD) or [l] (shared), then s^2, then
sigma^2, as derivatives with respect to these positive parameters.

Linear (Sec. 3 names it among the concrete kernels; no formula is printed):
the dot-product kernel k = s^2 x.x' (Rasmussen & Williams, ch. 4), whose only
parameter is s^2, so its gradient order is [s^2, sigma^2].

Sums (Sec. 3: the ``+`` composition of ``Scale``d kernels): SumKern holds
terms k_t, each with its own parameters and s_t^2, and one noise variance;
k = sum_t k_t, and its gradient order is each term's parameters without
sigma^2, in term order, then sigma^2.

Products (Sec. 3: ``*``): ProdKern holds factors k_f with unit outputscale
and one s^2 for the product, k = s^2 prod_f k_f; its gradient order is each
factor's parameters without s^2 and sigma^2, in factor order, then s^2, then
sigma^2.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import cho_factor, cho_solve

FAMILIES = ("rbf", "matern12", "matern32", "matern52", "periodic", "linear")


@dataclass
class Kern:
    """Kernel hyperparameters: family, lengthscale(s), outputscale s^2, noise sigma^2."""

    family: str
    lengthscale: object  # float (shared) or sequence of length d (ARD)
    outputscale: float = 1.0
    noise: float = 0.01
    period: float = 1.0  # the periodic family's period p (unused otherwise)
    ard: bool = field(init=False)

    def __post_init__(self):
        if self.family not in FAMILIES:
            raise ValueError(f"unknown family {self.family}")
        ls = np.asarray(self.lengthscale, dtype=np.float64)
        self.ard = ls.ndim == 1
        self.lengthscale = ls

    def ls_vec(self, d: int) -> np.ndarray:
        ls = np.asarray(self.lengthscale, dtype=np.float64)
        return np.full(d, float(ls)) if ls.ndim == 0 else ls.astype(np.float64)

    def n_params(self, d: int) -> int:
        if self.family == "linear":
            return 2
        return (d if self.ard else 1) + (3 if self.family == "periodic" else 2)

    def with_params(self, theta) -> "Kern":
        """New kernel from a parameter vector in gradient order."""
        theta = np.asarray(theta, dtype=np.float64)
        if self.family == "linear":
            return Kern("linear", self.lengthscale, float(theta[0]), float(theta[1]))
        extra = 3 if self.family == "periodic" else 2
        nl = len(theta) - extra
        ls = theta[:nl] if self.ard else float(theta[0])
        if self.family == "periodic":
            return Kern(self.family, ls, float(theta[nl + 1]), float(theta[nl + 2]), period=float(theta[nl]))
        return Kern(self.family, ls, float(theta[nl]), float(theta[nl + 1]))

    def params(self, d: int) -> np.ndarray:
        if self.family == "linear":
            return np.array([self.outputscale, self.noise])
        ls = self.ls_vec(d) if self.ard else np.array([float(self.lengthscale)])
        if self.family == "periodic":
            return np.concatenate([ls, [self.period, self.outputscale, self.noise]])
        return np.concatenate([ls, [self.outputscale, self.noise]])


class SumKern:
    """k = sum_t k_t with one noise variance (the ``+`` of Sec. 3 "Kernels").

    Each term is a Kern whose own noise is ignored.  Gradient order: the
    terms' parameters without sigma^2, in term order, then sigma^2."""

    family = "sum"

    def __init__(self, terms, noise: float):
        self.terms = list(terms)
        self.noise = float(noise)

    def n_params(self, d: int) -> int:
        return sum(t.n_params(d) - 1 for t in self.terms) + 1

    def params(self, d: int) -> np.ndarray:
        return np.concatenate([t.params(d)[:-1] for t in self.terms] + [[self.noise]])

    def with_params(self, theta) -> "SumKern":
        theta = np.asarray(theta, dtype=np.float64)
        out, off = [], 0
        for t in self.terms:
            m = len(t.params(_term_dim(t))) - 1
            out.append(t.with_params(np.concatenate([theta[off:off + m], [0.0]])))
            off += m
        return SumKern(out, float(theta[off]))


class ProdKern:
    """k = s^2 prod_f k_f (the ``*`` of Sec. 3 "Kernels"), factors at unit scale.

    A factor's own outputscale and noise are ignored.  Gradient order: every
    factor's parameters without s^2 and sigma^2, in factor order, then s^2,
    then sigma^2."""

    family = "prod"

    def __init__(self, factors, outputscale: float, noise: float):
        self.factors = [f.with_params(np.concatenate([f.params(_term_dim(f))[:-2], [1.0, 0.0]]))
                        for f in factors]
        self.outputscale = float(outputscale)
        self.noise = float(noise)

    def n_params(self, d: int) -> int:
        return sum(f.n_params(d) - 2 for f in self.factors) + 2

    def params(self, d: int) -> np.ndarray:
        return np.concatenate([f.params(d)[:-2] for f in self.factors] + [[self.outputscale, self.noise]])

    def with_params(self, theta) -> "ProdKern":
        theta = np.asarray(theta, dtype=np.float64)
        out, off = [], 0
        for f in self.factors:
            m = len(f.params(_term_dim(f))) - 2
            out.append(f.with_params(np.concatenate([theta[off:off + m], [1.0, 0.0]])))
            off += m
        return ProdKern(out, float(theta[off]), float(theta[off + 1]))


def _term_dim(t) -> int:
    """Input dimension implied by a term's lengthscales (1 for shared / linear)."""
    if hasattr(t, "factors"):
        return max(_term_dim(f) for f in t.factors)
    ls = np.asarray(t.lengthscale)
    return ls.shape[0] if ls.ndim == 1 else 1


# --------------------------------------------------------------------------
# Kernel entries (Sec. 3 "Kernels"; Sec. 2 defines K_ff, K_*f and K_y)
# --------------------------------------------------------------------------

def scaled_sqdist(X1: np.ndarray, X2: np.ndarray, ls: np.ndarray) -> np.ndarray:
    """r^2_ij = sum_k ((X1_ik - X2_jk) / l_k)^2 by direct differences, FP64."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    r2 = np.zeros((X1.shape[0], X2.shape[0]))
    for k in range(X1.shape[1]):
        dk = (X1[:, k, None] - X2[None, :, k]) / ls[k]
        r2 += dk * dk
    return r2


def shape_from_r2(family: str, r2: np.ndarray) -> np.ndarray:
    """Kernel profile f(r^2) with k = s^2 f (unit outputscale)."""
    if family == "rbf":
        return np.exp(-0.5 * r2)
    rho = np.sqrt(r2)
    if family == "matern12":
        return np.exp(-rho)
    if family == "matern32":
        a = math.sqrt(3.0) * rho
        return (1.0 + a) * np.exp(-a)
    if family == "matern52":
        a = math.sqrt(5.0) * rho
        return (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError(family)


def dshape_factor(family: str, r2: np.ndarray) -> np.ndarray:
    """g(r^2) such that d f / d l_k = g * Delta_k^2 / l_k^3 (unit outputscale).

    From d r^2 / d l_k = -2 Delta_k^2 / l_k^3 and the chain rule:
      RBF        g = exp(-r^2/2)
      Matern-1/2 g = exp(-rho) / rho            (limit 0 at rho = 0, see below)
      Matern-3/2 g = 3 exp(-sqrt3 rho)
      Matern-5/2 g = (5/3) (1 + sqrt5 rho) exp(-sqrt5 rho)
    For Matern-1/2 at rho = 0 every Delta_k is 0, so the product g Delta_k^2
    is 0; the factor is set to 0 there.
    """
    if family == "rbf":
        return np.exp(-0.5 * r2)
    rho = np.sqrt(r2)
    if family == "matern12":
        out = np.zeros_like(rho)
        nz = rho > 0
        out[nz] = np.exp(-rho[nz]) / rho[nz]
        return out
    if family == "matern32":
        return 3.0 * np.exp(-math.sqrt(3.0) * rho)
    if family == "matern52":
        a = math.sqrt(5.0) * rho
        return (5.0 / 3.0) * (1.0 + a) * np.exp(-a)
    raise ValueError(family)


def periodic_sum(X1: np.ndarray, X2: np.ndarray, ls: np.ndarray, period: float) -> np.ndarray:
    """S_ij = sum_k 2 sin^2(pi (X1_ik - X2_jk) / p) / l_k^2 (the periodic exponent)."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    S = np.zeros((X1.shape[0], X2.shape[0]))
    for k in range(X1.shape[1]):
        sk = np.sin(np.pi * (X1[:, k, None] - X2[None, :, k]) / period)
        S += 2.0 * sk * sk / ls[k] ** 2
    return S


def kernel_matrix(kern: Kern, X1: np.ndarray, X2: np.ndarray) -> np.ndarray:
    """K(X1, X2) with outputscale, no noise (Sec. 2: K_ff or K_*f).

    Periodic (Sec. 3 names it; the reading is the standard exp-sine-squared
    form with ARD lengthscales and one period, as in MacKay 1998 / Rasmussen
    & Williams eq. 4.31): k = s^2 exp(-sum_k 2 sin^2(pi (x_k - x'_k) / p) / l_k^2).
    """
    d = np.asarray(X1).shape[1]
    if kern.family == "sum":
        return sum(kernel_matrix(t, X1, X2) for t in kern.terms)
    if kern.family == "prod":
        K = kern.outputscale * np.ones((np.asarray(X1).shape[0], np.asarray(X2).shape[0]))
        for f in kern.factors:
            K = K * kernel_matrix(f, X1, X2)
        return K
    if kern.family == "linear":
        return kern.outputscale * (np.asarray(X1, dtype=np.float64) @ np.asarray(X2, dtype=np.float64).T)
    if kern.family == "periodic":
        return kern.outputscale * np.exp(-periodic_sum(X1, X2, kern.ls_vec(d), kern.period))
    r2 = scaled_sqdist(X1, X2, kern.ls_vec(d))
    return kern.outputscale * shape_from_r2(kern.family, r2)


def kernel_matrix_f32(kern: Kern, X1: np.ndarray, X2: np.ndarray, prescaled: bool = False) -> np.ndarray:
    """K(X1, X2) of an RBF or Matern kernel with every step of each entry in
    binary32 arithmetic, returned as FP64.

    prescaled=False evaluates the definition as written: differences, scaled
    squares, their sum, the profile and the outputscale.  prescaled=True
    evaluates the same kernel from coordinates scaled once per point, as an
    implementation that prescales its inputs does: with exp(z) = 2^(z log2 e),
    RBF is 2^(-|u - u'|^2) for u_k = x_k sqrt(log2(e) / 2) / l_k, and
    Matern-nu's e^(-sqrt(2 nu) rho) is 2^(-q) for q = |u - u'| with
    u_k = x_k sqrt(2 nu) log2(e) / l_k (its polynomial in sqrt(2 nu) rho =
    q ln 2).  The difference of two scaled coordinates is then rounded
    relative to the coordinates' magnitude, not the difference's, so its
    entries carry the larger error when |u| >> |u - u'| (small lengthscales
    against the data's range).

    Not a reference value: it differs from kernel_matrix by the binary32
    roundings of each entry, which is what an FP32 evaluation carries.  It
    sizes the floor that FP32 entries leave in FP64 checks (residuals,
    solutions, gradients) of an FP32-entry operator.
    """
    if kern.family not in ("rbf", "matern12", "matern32", "matern52"):
        raise ValueError(kern.family)
    f32 = np.float32
    X1 = np.asarray(X1, dtype=f32)
    X2 = np.asarray(X2, dtype=f32)
    d = X1.shape[1]
    ls = np.asarray(kern.ls_vec(d), dtype=np.float64)
    log2e = 1.0 / math.log(2.0)
    r2 = np.zeros((X1.shape[0], X2.shape[0]), dtype=f32)
    if not prescaled:
        ls32 = ls.astype(f32)
        for k in range(d):
            dk = (X1[:, k, None] - X2[None, :, k]) / ls32[k]
            r2 += dk * dk
        if kern.family == "rbf":
            prof = np.exp(f32(-0.5) * r2)
        else:
            rho = np.sqrt(r2)
            nu2 = {"matern12": 1.0, "matern32": 3.0, "matern52": 5.0}[kern.family]
            a = f32(math.sqrt(nu2)) * rho
            prof = _matern_poly32(kern.family, a) * np.exp(-a)
    else:
        c = math.sqrt(log2e / 2.0) if kern.family == "rbf" else \
            math.sqrt({"matern12": 1.0, "matern32": 3.0, "matern52": 5.0}[kern.family]) * log2e
        for k in range(d):
            sk = f32(c / ls[k])
            dk = X1[:, k, None] * sk - X2[None, :, k] * sk
            r2 += dk * dk
        if kern.family == "rbf":
            prof = np.exp2(-r2)
        else:
            q = np.sqrt(r2)
            prof = _matern_poly32(kern.family, q * f32(math.log(2.0))) * np.exp2(-q)
    return (f32(kern.outputscale) * prof.astype(f32)).astype(np.float64)


def _matern_poly32(family: str, a: np.ndarray) -> np.ndarray:
    """Matern polynomial in a = sqrt(2 nu) rho, binary32."""
    f32 = np.float32
    if family == "matern12":
        return np.ones_like(a)
    if family == "matern32":
        return f32(1.0) + a
    return f32(1.0) + a + a * a / f32(3.0)


def fp32_entry_floor(kern: Kern, X: np.ndarray, B: np.ndarray, Xsol: np.ndarray, rows, block: int = 256,
                     prescaled: bool = True):
    """Per column ||((K32 - K) Xsol)[rows]||_2 / ||B[rows]||_2: the part of an
    FP64-entry residual of Xsol that comes from evaluating the entries in
    binary32 (K32 from kernel_matrix_f32, by default in the prescaled form),
    over sampled rows."""
    X = np.asarray(X, dtype=np.float64)
    S = np.asarray(Xsol, dtype=np.float64).reshape(len(X), -1)
    Bm = np.asarray(B, dtype=np.float64).reshape(len(X), -1)
    rows = np.asarray(rows, dtype=np.int64)
    D = np.empty((len(rows), S.shape[1]))
    for b in range(0, len(rows), block):
        rb = rows[b:b + block]
        D[b:b + block] = (kernel_matrix_f32(kern, X[rb], X, prescaled) - kernel_matrix(kern, X[rb], X)) @ S
    return np.linalg.norm(D, axis=0) / np.linalg.norm(Bm[rows], axis=0)


def ky_matrix(kern: Kern, X: np.ndarray) -> np.ndarray:
    """K_y = K_ff + sigma^2 I (Sec. 2)."""
    K = kernel_matrix(kern, X, X)
    K[np.diag_indices_from(K)] += kern.noise
    return K


def ky_matvec(kern: Kern, X: np.ndarray, V: np.ndarray) -> np.ndarray:
    """K_y V in FP64, the product CG needs (Sec. 2 "CG-based inference")."""
    V = np.asarray(V, dtype=np.float64)
    return ky_matrix(kern, X) @ V


def ky_matvec_rows(kern: Kern, X: np.ndarray, V: np.ndarray, rows, block: int = 256) -> np.ndarray:
    """Selected rows of K_y V without forming K (sampled check at large N).

    out[r] = s^2 sum_j k(x_r, x_j) V_j + sigma^2 V_r, accumulated in FP64 over
    row blocks so memory stays O(block * N).
    """
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    V2 = V.reshape(V.shape[0], -1)
    out = np.empty((len(rows), V2.shape[1]))
    for b in range(0, len(rows), block):
        rb = rows[b:b + block]
        K = kernel_matrix(kern, X[rb], X)
        out[b:b + block] = K @ V2 + kern.noise * V2[rb]
    return out.reshape((len(rows),) + V.shape[1:])


def cross_matvec_blocked(kern: Kern, Xs: np.ndarray, X: np.ndarray, a: np.ndarray,
                         block: int = 512) -> np.ndarray:
    """K(Xs, X) a accumulated over row blocks of Xs (O(block * N) memory)."""
    a = np.asarray(a, dtype=np.float64)
    out = np.empty((Xs.shape[0],) + a.shape[1:])
    for b in range(0, Xs.shape[0], block):
        out[b:b + block] = kernel_matrix(kern, Xs[b:b + block], X) @ a
    return out


# --------------------------------------------------------------------------
# Exact inference (Sec. 2: mean, MLL; "Exact inference via Cholesky")
# --------------------------------------------------------------------------

def cholesky(kern: Kern, X: np.ndarray):
    return cho_factor(ky_matrix(kern, X), lower=True)


def solve(kern: Kern, X: np.ndarray, B: np.ndarray, chol=None) -> np.ndarray:
    """K_y^{-1} B by Cholesky (LAPACK dpotrf / dpotrs through scipy)."""
    c = chol if chol is not None else cholesky(kern, X)
    return cho_solve(c, np.asarray(B, dtype=np.float64))


def predict_mean(kern: Kern, X: np.ndarray, Xs: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """mu_* = K_*f alpha with alpha = K_y^{-1} y (Sec. 2)."""
    return kernel_matrix(kern, Xs, X) @ np.asarray(alpha, dtype=np.float64)


def logdet(kern: Kern, X: np.ndarray, chol=None) -> float:
    c = chol if chol is not None else cholesky(kern, X)
    return 2.0 * float(np.sum(np.log(np.diag(c[0]))))


def mll(kern: Kern, X: np.ndarray, y: np.ndarray) -> float:
    """log p(y|X) = -1/2 [y^T K_y^{-1} y + log|K_y| + N log 2 pi] (Sec. 2)."""
    y = np.asarray(y, dtype=np.float64)
    c = cholesky(kern, X)
    alpha = cho_solve(c, y)
    n = y.shape[0]
    return -0.5 * (float(y @ alpha) + logdet(kern, X, c) + n * math.log(2.0 * math.pi))


def dky_matrices(kern: Kern, X: np.ndarray):
    """dK_y/dtheta for theta in gradient order, as dense FP64 matrices.

    d/dl_k : s^2 g(r^2) Delta_k^2 / l_k^3   (summed over k for a shared l)
    d/ds^2 : K / s^2 = f(r^2)
    d/dsigma^2 : I
    The periodic family has d/dp between the lengthscales and s^2.
    """
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    if kern.family == "sum":
        # d(sum_t k_t)/d theta_t = d k_t / d theta_t; sigma^2 once at the end
        mats = []
        for t in kern.terms:
            mats += dky_matrices(t, X)[:-1]
        mats.append(np.eye(n))
        return mats
    if kern.family == "prod":
        # d(s^2 prod_f k_f)/d theta_f = s^2 (d k_f / d theta_f) prod_{g != f} k_g
        Ks = [kernel_matrix(f, X, X) for f in kern.factors]
        mats = []
        for i, f in enumerate(kern.factors):
            others = np.ones((n, n))
            for j, Kg in enumerate(Ks):
                if j != i:
                    others = others * Kg
            mats += [kern.outputscale * dK * others for dK in dky_matrices(f, X)[:-2]]
        prod = np.ones((n, n))
        for Kg in Ks:
            prod = prod * Kg
        mats.append(prod)
        mats.append(np.eye(n))
        return mats
    if kern.family == "linear":
        # k = s^2 x.x': d/ds^2 = x.x'
        return [X @ X.T, np.eye(n)]
    ls = kern.ls_vec(d)
    if kern.family == "periodic":
        # k = s^2 exp(-S), S = sum_k 2 sin^2(pi D_k / p) / l_k^2:
        # dk/dl_k = k 4 sin^2(pi D_k / p) / l_k^3
        # dk/dp   = k sum_k (2 pi D_k / (p^2 l_k^2)) sin(2 pi D_k / p)
        p = kern.period
        K = kernel_matrix(kern, X, X)
        per_dim, dp = [], np.zeros((n, n))
        for k in range(d):
            dk = X[:, k, None] - X[None, :, k]
            sk = np.sin(np.pi * dk / p)
            per_dim.append(K * 4.0 * sk * sk / ls[k] ** 3)
            dp += 2.0 * np.pi * dk / (p * p * ls[k] ** 2) * np.sin(2.0 * np.pi * dk / p)
        mats = per_dim if kern.ard else [sum(per_dim)]
        mats.append(K * dp)
        mats.append(K / kern.outputscale)
        mats.append(np.eye(n))
        return mats
    r2 = scaled_sqdist(X, X, ls)
    g = kern.outputscale * dshape_factor(kern.family, r2)
    per_dim = []
    for k in range(d):
        dk = X[:, k, None] - X[None, :, k]
        per_dim.append(g * dk * dk / ls[k] ** 3)
    mats = per_dim if kern.ard else [sum(per_dim)]
    mats.append(shape_from_r2(kern.family, r2))
    mats.append(np.eye(n))
    return mats


def mll_grad(kern: Kern, X: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Exact gradient of the MLL: 1/2 a^T dK a - 1/2 tr(K_y^{-1} dK), a = K_y^{-1} y.

    The trace is taken as sum_ij (K_y^{-1})_ij (dK)_ij (both symmetric).
    """
    y = np.asarray(y, dtype=np.float64)
    c = cholesky(kern, X)
    a = cho_solve(c, y)
    Kinv = cho_solve(c, np.eye(len(y)))
    out = []
    for dK in dky_matrices(kern, X):
        out.append(0.5 * float(a @ dK @ a) - 0.5 * float(np.sum(Kinv * dK)))
    return np.array(out)


def same_probe_grad(kern: Kern, X: np.ndarray, y: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """The stochastic-trace gradient estimator evaluated exactly for given probes.

    g_theta = 1/2 a^T dK a - 1/2 (1/p) sum_c u_c^T dK z_c,  u_c = K_y^{-1} z_c,
    i.e. tr(K_y^{-1} dK) replaced by its Hutchinson estimate with the probes Z
    (Rademacher, Sec. 4.3), with every solve exact (Cholesky).
    """
    y = np.asarray(y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    p = Z.shape[1]
    c = cholesky(kern, X)
    a = cho_solve(c, y)
    U = cho_solve(c, Z)
    out = []
    for dK in dky_matrices(kern, X):
        out.append(0.5 * float(a @ dK @ a) - 0.5 / p * float(np.sum(U * (dK @ Z))))
    return np.array(out)


def adjoint_bilinear(kern: Kern, X: np.ndarray, A: np.ndarray, B: np.ndarray,
                     colw) -> np.ndarray:
    """sum_c colw_c A_c^T (dK_y/dtheta) B_c for every theta (vector-Jacobian product)."""
    A = np.asarray(A, dtype=np.float64).reshape(len(X), -1)
    B = np.asarray(B, dtype=np.float64).reshape(len(X), -1)
    colw = np.asarray(colw, dtype=np.float64)
    return np.array([float(np.sum((A * colw) * (dK @ B))) for dK in dky_matrices(kern, X)])


def solve_residual(kern: Kern, X: np.ndarray, B: np.ndarray, Xsol: np.ndarray, rows=None) -> np.ndarray:
    """Per-column ||B - K_y Xsol||_2 / ||B||_2 in FP64 (optionally over sampled rows)."""
    B = np.asarray(B, dtype=np.float64).reshape(len(X), -1)
    S = np.asarray(Xsol, dtype=np.float64).reshape(len(X), -1)
    if rows is None:
        R = B - ky_matvec(kern, X, S)
        return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
    R = B[rows] - ky_matvec_rows(kern, X, S, rows)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(B[rows], axis=0)
