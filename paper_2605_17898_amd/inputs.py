"""Seeded synthetic GP workloads.

This module only draws inputs: training points, targets, test points and
probe matrices.  It holds none of the method's arithmetic and is shared by the
HIP path's tests and benchmark and by the oracle checks, so both sides see the
identical float32 arrays.

Workloads (all synthetic; the paper's accuracy datasets are not used):

* ``exact1k``   N=1024, d=2, X ~ U[0,1]^2, y = sin(2 pi x1) cos(2 pi x2) + N(0, 0.1^2),
                RBF l=0.2, s^2=1, sigma^2=0.01.
* ``matern20k`` N=20000, d=3, X ~ N(0, I), y = sum_k sin(x_k) + N(0, 0.05^2),
                Matern-5/2 l=1, s^2=1, sigma^2=0.01; 2000 test points ~ N(0, I).
* ``rbf100k``   N=100000, d=4, X ~ U[-1,1]^4, y = sum_k sin(pi x_k) + N(0, 0.1^2),
                RBF l=0.3, s^2=1, sigma^2=0.01; 32 Rademacher probes (t = 33).
* ``batch64``   64 problems, N_b ~ U{2000..30000}, d_b ~ U{1..6}, ARD RBF with
                l ~ U[0.1, 1]^d_b, X_b ~ U[0,1]^d_b, y = sum_k sin(2 pi x_k) + N(0, 0.1^2),
                s^2=1, sigma^2=0.01, 16 probes.
* ``rbf500k``   N=500000, d=2, X ~ U[0,1]^2, y = sin(6 x1) + cos(4 x2) + N(0, 0.1^2),
                RBF l=0.05, s^2=1, sigma^2=0.01, 16 probes.

Seeds: workload k (1..5 in the order above) draws X then the noise from
``default_rng(100 + k)``, test points from ``default_rng(200 + k)`` and probes
from ``default_rng(300 + k)``; problem b of the batch draws its sizes from
``default_rng(10_000 + b)``.  ``n`` overrides shrink a workload while keeping
its distribution, lengthscale and noise (the smaller parity cases).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

FAMILY_IDS = {"rbf": 0, "matern12": 1, "matern32": 2, "matern52": 3}


@dataclass
class Workload:
    name: str
    X: np.ndarray                 # [n, d] float32
    y: np.ndarray                 # [n] float32
    family: str
    lengthscale: object           # float or float32 array [d]
    outputscale: float
    noise: float
    Z: Optional[np.ndarray] = None   # [n, p] float32 Rademacher probes
    Xs: Optional[np.ndarray] = None  # [m, d] float32 test points
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]


def rademacher(rng: np.random.Generator, n: int, p: int) -> np.ndarray:
    """n x p matrix of independent +-1 entries, probability 1/2 each (float32)."""
    return (2.0 * rng.integers(0, 2, size=(n, p)) - 1.0).astype(np.float32)


def gaussian_rhs(seed: int, n: int, t: int) -> np.ndarray:
    """n x t float32 standard-normal right-hand sides."""
    return np.random.default_rng(seed).standard_normal((n, t)).astype(np.float32)


def exact1k(n: int = 1024, probes: int = 0) -> Workload:
    rng = np.random.default_rng(101)
    X = rng.uniform(0.0, 1.0, size=(n, 2))
    y = np.sin(2 * np.pi * X[:, 0]) * np.cos(2 * np.pi * X[:, 1]) + 0.1 * rng.standard_normal(n)
    w = Workload("exact1k", X.astype(np.float32), y.astype(np.float32), "rbf", 0.2, 1.0, 0.01)
    if probes:
        w.Z = rademacher(np.random.default_rng(301), n, probes)
    return w


def matern20k(n: int = 20000, m: int = 2000, probes: int = 0) -> Workload:
    rng = np.random.default_rng(102)
    X = rng.standard_normal((n, 3))
    y = np.sin(X).sum(axis=1) + 0.05 * rng.standard_normal(n)
    Xs = np.random.default_rng(202).standard_normal((m, 3))
    w = Workload("matern20k", X.astype(np.float32), y.astype(np.float32), "matern52", 1.0, 1.0, 0.01,
                 Xs=Xs.astype(np.float32))
    if probes:
        w.Z = rademacher(np.random.default_rng(302), n, probes)
    return w


def rbf100k(n: int = 100000, probes: int = 32, m: int = 2000) -> Workload:
    rng = np.random.default_rng(103)
    X = rng.uniform(-1.0, 1.0, size=(n, 4))
    y = np.sin(np.pi * X).sum(axis=1) + 0.1 * rng.standard_normal(n)
    Xs = np.random.default_rng(203).uniform(-1.0, 1.0, size=(m, 4))
    w = Workload("rbf100k", X.astype(np.float32), y.astype(np.float32), "rbf", 0.3, 1.0, 0.01,
                 Xs=Xs.astype(np.float32))
    if probes:
        w.Z = rademacher(np.random.default_rng(303), n, probes)
    return w


def batch_problem(b: int, n: Optional[int] = None, probes: int = 16) -> Workload:
    rng = np.random.default_rng(10_000 + b)
    nb = int(rng.integers(2000, 30001))
    db = int(rng.integers(1, 7))
    ls = rng.uniform(0.1, 1.0, size=db)
    if n is not None:
        nb = n
    X = rng.uniform(0.0, 1.0, size=(nb, db))
    y = np.sin(2 * np.pi * X).sum(axis=1) + 0.1 * rng.standard_normal(nb)
    w = Workload(f"batch64[{b}]", X.astype(np.float32), y.astype(np.float32), "rbf",
                 ls.astype(np.float32), 1.0, 0.01)
    if probes:
        w.Z = rademacher(np.random.default_rng(304 * 1000 + b), nb, probes)
    return w


def batch_sizes(count: int = 64):
    """(N_b, d_b) of every batch problem without drawing its data."""
    out = []
    for b in range(count):
        rng = np.random.default_rng(10_000 + b)
        out.append((int(rng.integers(2000, 30001)), int(rng.integers(1, 7))))
    return out


def batch64(count: int = 64, n: Optional[int] = None, probes: int = 16):
    return [batch_problem(b, n=n, probes=probes) for b in range(count)]


def rbf500k(n: int = 500000, probes: int = 16) -> Workload:
    rng = np.random.default_rng(105)
    X = rng.uniform(0.0, 1.0, size=(n, 2))
    y = np.sin(6 * X[:, 0]) + np.cos(4 * X[:, 1]) + 0.1 * rng.standard_normal(n)
    w = Workload("rbf500k", X.astype(np.float32), y.astype(np.float32), "rbf", 0.05, 1.0, 0.01)
    if probes:
        w.Z = rademacher(np.random.default_rng(305), n, probes)
    return w


def ski200k(n: int = 200000, d: int = 1) -> Workload:
    """N = 200000 points for the structured-interpolation path (the paper's SKI
    scale, D = 1): uniform on [0, 1]^d, a smooth signal plus noise, RBF."""
    rng = np.random.default_rng(106)
    X = rng.uniform(0.0, 1.0, size=(n, d))
    y = np.sin(8 * np.pi * X).sum(axis=1) + 0.1 * rng.standard_normal(n)
    return Workload(f"ski200k_d{d}", X.astype(np.float32), y.astype(np.float32), "rbf", 0.05, 1.0, 0.01)


def random_problem(seed: int, n: int, d: int, family: str = "rbf", ard: bool = False,
                   dist: str = "uniform", lengthscale=None, outputscale: float = 1.3,
                   noise: float = 0.05) -> Workload:
    """Generic seeded problem for parity sweeps over (family, d, ARD, n)."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        X = rng.uniform(0.0, 1.0, size=(n, d))
    else:
        X = rng.standard_normal((n, d))
    if lengthscale is None:
        lengthscale = rng.uniform(0.15, 0.6, size=d).astype(np.float32) if ard else 0.35
    y = np.sin(3.0 * X).sum(axis=1) + 0.1 * rng.standard_normal(n)
    return Workload(f"random[{seed}]", X.astype(np.float32), y.astype(np.float32), family,
                    lengthscale, outputscale, noise)
