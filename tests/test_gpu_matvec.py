"""Parity of the HIP matrix-free K_y V against the FP64 oracle.

Bar: per-column ||out - ref||_2 / ||ref||_2 <= 1e-5 for the FP32 form, at
sizes that span several 256-row blocks with a ragged tail, and on sampled
rows at the full 100k and 500k workloads in the launch configuration the
benchmark uses.
"""

import math

import numpy as np
import pytest
import torch

from oracle import gp
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, col_rel_err, dev, host, mkern, okern

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


def _rhs(kind, X, t, seed):
    n = X.shape[0]
    if kind == "normal":
        return inputs.gaussian_rhs(seed, n, t)
    if kind == "ones":
        return np.ones((n, t), np.float32)
    return np.repeat(np.sin(3.0 * X[:, :1]), t, axis=1).astype(np.float32)


@pytest.mark.parametrize("family", ["rbf", "matern12", "matern32", "matern52"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
def test_matvec_families_dims(mf, family, d):
    banner(f"matvec family={family} d={d} n=1000 t=3")
    w = inputs.random_problem(40 + d, 1000, d, family, ard=(d % 2 == 0))
    V = _rhs("normal", w.X, 3, d)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V)))
    ref = gp.ky_matvec(okern(w), w.X, V)
    assert col_rel_err(out, ref).max() <= TOL


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 7, 8, 9, 16, 17, 20, 32, 33, 40, 65])
def test_matvec_column_counts(mf, t):
    banner(f"matvec rbf d=4 n=1537 t={t}")
    w = inputs.rbf100k(n=1537, probes=0)
    V = _rhs("normal", w.X, t, t)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V)))
    ref = gp.ky_matvec(okern(w), w.X, V)
    assert col_rel_err(out, ref).max() <= TOL


@pytest.mark.parametrize("t", [16, 17, 33, 49, 64])
@pytest.mark.parametrize("family", ["rbf", "matern52"])
def test_matvec_mfma_contraction_and_valu_forms(mf, t, family):
    # FP32 moves 16-column tiles of the contraction onto FP32 MFMA for these t;
    # the explicit VALU-only form must agree with the oracle just the same.
    banner(f"matvec fp32 (MFMA contraction) and fp32_valu family={family} t={t} n=2113")
    w = inputs.random_problem(60 + t, 2113, 4, family, ard=True, noise=0.02)
    V = inputs.gaussian_rhs(t + 1, w.n, t)
    ref = gp.ky_matvec(okern(w), w.X, V)
    a = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="fp32"))
    b = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision="fp32_valu"))
    assert col_rel_err(a, ref).max() <= TOL
    assert col_rel_err(b, ref).max() <= TOL


@pytest.mark.parametrize("n", [1, 2, 63, 255, 256, 257, 4097])
@pytest.mark.parametrize("kind", ["normal", "ones", "smooth"])
def test_matvec_ragged_sizes(mf, n, kind):
    banner(f"matvec exact1k geometry n={n} v={kind}")
    w = inputs.exact1k(n=n)
    V = _rhs(kind, w.X, 2, n)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V)))
    ref = gp.ky_matvec(okern(w), w.X, V)
    assert col_rel_err(out, ref).max() <= TOL


def test_matvec_vector_shape_and_zero_noise(mf):
    banner("matvec 1-d vector, sigma^2 = 0")
    w = inputs.matern20k(n=3000)
    w.noise = 0.0
    v = _rhs("normal", w.X, 1, 5)[:, 0].copy()
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(v)))
    ref = gp.ky_matvec(okern(w), w.X, v)
    assert out.shape == v.shape
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) <= TOL


def test_matvec_special_structures(mf):
    banner("matvec far-apart and identical points")
    n = 300
    Xfar = (np.arange(n, dtype=np.float32)[:, None] * 100.0).repeat(2, axis=1)
    v = _rhs("normal", Xfar, 1, 9)
    for fam in ("rbf", "matern12", "matern32", "matern52"):
        k = mf.Kernel(fam, 0.5, 1.5, 0.1)
        out = host(mf.kernel_matvec(k, dev(Xfar), dev(v)))
        np.testing.assert_allclose(out, 1.6 * v, rtol=1e-6)
    Xsame = np.full((n, 3), 0.25, np.float32)
    for fam in ("rbf", "matern52"):
        k = mf.Kernel(fam, 0.5, 0.8, 0.05)
        out = host(mf.kernel_matvec(k, dev(Xsame), dev(v)))
        ref = 0.05 * v.astype(np.float64) + 0.8 * v.astype(np.float64).sum()
        assert col_rel_err(out, ref).max() <= TOL


def test_matvec_deterministic(mf):
    banner("matvec bitwise determinism")
    w = inputs.rbf100k(n=20000, probes=4)
    V = np.concatenate([w.y[:, None], w.Z], axis=1)
    a = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V)))
    b = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V)))
    assert np.array_equal(a, b)


def test_matvec_full_rbf100k_sampled_rows(mf):
    # The benchmark's workload and launch: n = 100000, d = 4, t = 33 = [y, 32 probes].
    banner("matvec rbf100k full size t=33, 2048 sampled rows")
    w = inputs.rbf100k()
    V = np.concatenate([w.y[:, None], w.Z], axis=1)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V)))
    rows = np.random.default_rng(7).choice(w.n, size=2048, replace=False)
    ref = gp.ky_matvec_rows(okern(w), w.X, V, rows)
    assert col_rel_err(out[rows], ref).max() <= TOL
    assert np.isfinite(out).all()


def test_matvec_full_rbf500k_sampled_rows(mf):
    banner("matvec rbf500k full size t=17, 512 sampled rows")
    w = inputs.rbf500k()
    V = np.concatenate([w.y[:, None], w.Z], axis=1)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V)))
    rows = np.random.default_rng(8).choice(w.n, size=512, replace=False)
    ref = gp.ky_matvec_rows(okern(w), w.X, V, rows)
    assert col_rel_err(out[rows], ref).max() <= TOL


def test_rademacher_bit_exact(mf):
    from oracle import probes
    banner("rademacher probes vs SplitMix64 oracle")
    for seed, n, p in [(0, 100, 3), (303, 4097, 17), (2 ** 63 + 5, 1000, 1)]:
        Z = host(mf.rademacher(seed, n, p))
        assert np.array_equal(Z, probes.rademacher(seed, n, p).astype(np.float32))
