"""K_y V of the HIP path against the FP64 oracle over seeded random shapes.

The targeted tests pin each kernel at chosen shapes; this sweep draws
(family, d, ARD, n, t, product form) from a fixed seed, so that the
combinations in between (tiny and ragged n, column counts that split into
blocks, every form on every family) are exercised too.  The bar per form is
the one the targeted tests use: FP32 forms and BF16-x3 1e-5 per column
(relative 2-norm), BF16-x2 3e-5.
"""

import numpy as np
import pytest

from oracle import gp
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, col_rel_err, dev, host, mkern, okern

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp32_direct": 1e-5, "fp32_valu": 1e-5, "fp32_gram": 1e-5, "bf16x2": 3e-5, "bf16x3": 1e-5}
FAMILIES = ["rbf", "matern12", "matern32", "matern52"]


def _cases(count=36, seed=20261203):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        family = FAMILIES[k % 4]
        forms = ["fp32", "fp32_direct", "fp32_valu", "bf16x2", "bf16x3"] + (["fp32_gram"] if family == "rbf" else [])
        form = forms[int(rng.integers(len(forms)))]
        d = int(rng.integers(1, 9))
        n = int(rng.choice([int(rng.integers(1, 40)), int(rng.integers(40, 1200)), int(rng.integers(1200, 5000))]))
        t = int(rng.choice([int(rng.integers(1, 9)), int(rng.integers(9, 40)), int(rng.integers(40, 65))]))
        out.append((k, family, d, bool(rng.integers(2)), n, t, form))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}-{c[1]}-d{c[2]}-n{c[4]}-t{c[5]}-{c[6]}")
def test_matvec_random_shape(mf, case):
    k, family, d, ard, n, t, form = case
    banner(f"matvec random shape #{k}: {family} d={d} ard={ard} n={n} t={t} {form}")
    w = inputs.random_problem(700 + k, n, d, family, ard=ard, noise=0.04)
    V = inputs.gaussian_rhs(800 + k, n, t)
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision=form))
    ref = gp.ky_matrix(okern(w), w.X) @ V.astype(np.float64)
    err = col_rel_err(out.reshape(n, t), ref.reshape(n, t))
    assert err.max() <= TOL[form], (err.max(), case)


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


def _cg_cases(count=12, seed=20261204):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        family = FAMILIES[k % 4]
        form = ["fp32", "fp32_direct", "bf16x3"][k % 3]
        d = int(rng.integers(1, 7))
        n = int(rng.integers(150, 3000))
        t = int(rng.integers(1, 10))
        out.append((k, family, d, bool(rng.integers(2)), n, t, form))
    return out


@pytest.mark.parametrize("case", _cg_cases(), ids=lambda c: f"{c[0]}-{c[1]}-d{c[2]}-n{c[4]}-t{c[5]}-{c[6]}")
def test_cg_random_shape(mf, case):
    # Every column to the recomputed 1e-6, and the oracle's FP64-entry
    # residual of the returned solution within that 1e-6 plus the part the
    # FP32 entries leave (computed by the oracle, factor 2 for its own
    # binary32 rounding order), on every row.
    k, family, d, ard, n, t, form = case
    banner(f"cg random shape #{k}: {family} d={d} ard={ard} n={n} t={t} {form}")
    w = inputs.random_problem(900 + k, n, d, family, ard=ard, noise=0.04)
    B = np.concatenate([w.y[:, None], inputs.gaussian_rhs(950 + k, n, t - 1)], axis=1)
    x, info, _, st = mf.cg_solve(mkern(w), dev(w.X), dev(B), tol=1e-6, precision=form)
    assert st == mf.OK, info
    assert max(i["rel_resid_true"] for i in info) <= 1e-6
    xs = host(x).reshape(n, t)
    rows = np.arange(n)
    res = gp.solve_residual(okern(w), w.X, B, xs, rows=rows)
    floor = gp.fp32_entry_floor(okern(w), w.X, B, xs, rows)
    assert np.all(res <= 2 * floor + 2e-6), (res, floor, case)


@pytest.mark.parametrize("family", FAMILIES)
@pytest.mark.parametrize("form", ["fp32", "fp32_valu"])
def test_kernel_entries_match_binary32_model(mf, family, form):
    # Columns of K itself (V = the first 64 unit vectors) against the oracle's
    # binary32 model of the same prescaled evaluation: both round every step
    # to binary32, so entries agree to a few ulp wherever the entry is not
    # negligible.  A wrong constant in an entry's formula (a coefficient of
    # the Matern polynomial, a prescale factor) shows here as a systematic
    # relative difference even where the column bar of the products hides it.
    banner(f"kernel entries vs binary32 model: {family} {form}")
    w = inputs.random_problem(990, 512, 3, family, ard=True, noise=0.04)
    V = np.zeros((w.n, 64), dtype=np.float32)
    V[np.arange(64), np.arange(64)] = 1.0
    out = host(mf.kernel_matvec(mkern(w), dev(w.X), dev(V), precision=form)).astype(np.float64)
    k = okern(w)
    Kg = (out - k.noise * V.astype(np.float64)) / k.outputscale
    Km = gp.kernel_matrix_f32(gp.Kern(family, w.lengthscale, 1.0, 0.0), w.X, w.X[:64], prescaled=True)
    big = Km > 1e-6
    rel = np.abs(Kg[big] - Km[big]) / Km[big]
    print(f"{family} {form}: max relative entry difference {rel.max():.2e} over {big.sum()} entries")
    assert rel.max() <= 2e-6
