"""Plain FP64 CPU oracle for the matrix-free Gaussian-process path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything in this directory; only the tests, the smoke check and the
benchmark's ``cpu_baseline`` leg do.  The oracle forms K explicitly, solves
with Cholesky and evaluates every stochastic estimator exactly, so that the
HIP path can be checked against plain definitions (LightGP, Sec. 2
"Background": predictive mean, predictive covariance and the log marginal
likelihood; Sec. 3 "Library Design": the kernel families and the CG /
stochastic-Lanczos solver).

Modules
-------
gp       kernel entries, K_y products, Cholesky solve, predictive mean,
         log marginal likelihood and its exact and same-probe gradients.
krylov   plain FP64 conjugate gradients, Lanczos with full
         reorthogonalisation, the CG-to-Lanczos coefficient map and the
         Gauss-quadrature log-determinant.
brute    pure-Python double loops for tiny inputs.
probes   the counter-based Rademacher probe generator (SplitMix64).
bf16     round-to-nearest-even bfloat16 and the BF16 tile-product models.
precond  rank-k pivoted Cholesky, the Woodbury preconditioner, preconditioned
         CG and the preconditioned log-determinant and gradient estimators.
variance the exact predictive variance and its stochastic diagonal
         estimator (Rademacher probes).
ski      structured kernel interpolation: the regular grid, cubic
         convolution weights and the dense W K_UU W^T products.
"""

from . import gp, krylov, brute, probes, bf16, precond, variance, ski  # noqa: F401
