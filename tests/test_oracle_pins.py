"""Pins for the FP64 oracle: closed forms, brute force, library routines, invariants.

Each check ties the oracle to something other than itself, so that a dropped
term, a wrong sign or index or a transposed operand in it fails here.
"""

import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats
import torch

from oracle import bf16, brute, gp, krylov, probes
from paper_2605_17898_amd import inputs

# the four families that decay with distance (the periodic family has its own
# pins in test_oracle_periodic.py)
FAMS = ("rbf", "matern12", "matern32", "matern52")
HERE = os.path.dirname(os.path.abspath(__file__))


def _pts(seed, n, d, scale=1.0):
    return np.random.default_rng(seed).uniform(0, scale, size=(n, d))


# ---------------------------------------------------------------- entries

@pytest.mark.parametrize("s2", [1.0, 2.5])
def test_entry_closed_forms(s2):
    e = math.exp(-1.0)
    x0 = np.zeros((1, 1))
    # k(x, x) = s^2 for every family
    for f in FAMS:
        assert gp.kernel_matrix(gp.Kern(f, 0.7, s2), x0, x0)[0, 0] == pytest.approx(s2, rel=1e-15)
    # RBF at r^2 = 2 (distance sqrt2 * l): s^2 e^-1
    l = 0.4
    k = gp.kernel_matrix(gp.Kern("rbf", l, s2), x0, np.array([[math.sqrt(2.0) * l]]))[0, 0]
    assert k == pytest.approx(s2 * e, rel=1e-14)
    # Matern-1/2 at rho = 1: s^2 e^-1
    k = gp.kernel_matrix(gp.Kern("matern12", l, s2), x0, np.array([[l]]))[0, 0]
    assert k == pytest.approx(s2 * e, rel=1e-14)
    # Matern-3/2 at sqrt3 rho = 1: s^2 (1 + 1) e^-1
    k = gp.kernel_matrix(gp.Kern("matern32", l, s2), x0, np.array([[l / math.sqrt(3.0)]]))[0, 0]
    assert k == pytest.approx(2.0 * s2 * e, rel=1e-14)
    # Matern-5/2 at sqrt5 rho = 1: s^2 (1 + 1 + 1/3) e^-1 = (7/3) s^2 e^-1
    k = gp.kernel_matrix(gp.Kern("matern52", l, s2), x0, np.array([[l / math.sqrt(5.0)]]))[0, 0]
    assert k == pytest.approx(7.0 / 3.0 * s2 * e, rel=1e-14)


def test_ard_scales_each_dimension():
    # ARD: an offset of l_k along axis k alone gives r^2 = 1 whatever k is.
    ls = np.array([0.2, 0.5, 1.3])
    for k in range(3):
        x1 = np.zeros((1, 3))
        x1[0, k] = ls[k]
        val = gp.kernel_matrix(gp.Kern("rbf", ls, 1.0), np.zeros((1, 3)), x1)[0, 0]
        assert val == pytest.approx(math.exp(-0.5), rel=1e-14)


@pytest.mark.parametrize("family", FAMS)
@pytest.mark.parametrize("ard", [False, True])
def test_matvec_vs_brute_force(family, ard):
    rng = np.random.default_rng(7)
    n, d, t = 37, 3, 2
    X = rng.uniform(0, 1, size=(n, d))
    V = rng.standard_normal((n, t))
    ls = rng.uniform(0.2, 0.7, size=d) if ard else 0.45
    kern = gp.Kern(family, ls, 1.7, 0.03)
    ref = np.array(brute.ky_matvec(family, X.tolist(), V.tolist(), list(kern.ls_vec(d)), 1.7, 0.03))
    np.testing.assert_allclose(gp.ky_matvec(kern, X, V), ref, rtol=1e-13, atol=1e-13)
    rows = np.array([0, 5, 36])
    np.testing.assert_allclose(gp.ky_matvec_rows(kern, X, V, rows, block=2), ref[rows], rtol=1e-13)


@pytest.mark.parametrize("family", FAMS)
def test_operator_invariants(family):
    rng = np.random.default_rng(3)
    n, d = 120, 2
    X = rng.uniform(0, 1, size=(n, d))
    kern = gp.Kern(family, 0.3, 1.2, 0.02)
    Ky = gp.ky_matrix(kern, X)
    assert np.array_equal(Ky, Ky.T)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    assert u @ gp.ky_matvec(kern, X, v) == pytest.approx(v @ gp.ky_matvec(kern, X, u), rel=1e-12)
    # v^T K_y v >= sigma^2 ||v||^2 (K is PSD)
    assert v @ gp.ky_matvec(kern, X, v) >= 0.02 * (v @ v) * (1 - 1e-12)
    assert np.linalg.eigvalsh(Ky).min() >= 0.02 * (1 - 1e-9)
    # permutation equivariance
    perm = rng.permutation(n)
    np.testing.assert_allclose(gp.ky_matvec(kern, X[perm], v[perm]), gp.ky_matvec(kern, X, v)[perm],
                               rtol=1e-12, atol=1e-12)
    # linearity
    np.testing.assert_allclose(gp.ky_matvec(kern, X, 2 * u - 3 * v),
                               2 * gp.ky_matvec(kern, X, u) - 3 * gp.ky_matvec(kern, X, v),
                               rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------- special cases

@pytest.mark.parametrize("family", FAMS)
def test_far_apart_points(family):
    # points spaced far beyond the lengthscale: every off-diagonal entry is 0
    n = 12
    X = np.arange(n, dtype=float)[:, None] * 1e3
    kern = gp.Kern(family, 0.5, 1.5, 0.1)
    y = np.random.default_rng(1).standard_normal(n)
    np.testing.assert_array_equal(gp.ky_matrix(kern, X), 1.6 * np.eye(n))
    np.testing.assert_allclose(gp.solve(kern, X, y), y / 1.6, rtol=1e-14)
    assert gp.logdet(kern, X) == pytest.approx(n * math.log(1.6), rel=1e-14)
    # CG reaches the solution after one step; SLQ is exact at m = 1
    x, al, be, it = krylov.cg(lambda V: gp.ky_matvec(kern, X, V), y, tol=1e-14)
    assert it[0] == 1
    np.testing.assert_allclose(x, y / 1.6, rtol=1e-14)
    z = np.sign(np.random.default_rng(2).standard_normal(n))
    _, q, _ = krylov.slq_logdet(lambda V: gp.ky_matvec(kern, X, V), z[:, None], tol=1e-14)
    assert q[0] == pytest.approx(n * math.log(1.6), rel=1e-13)


@pytest.mark.parametrize("family", FAMS)
def test_identical_points(family):
    # K_y = sigma^2 I + s^2 1 1^T: Sherman-Morrison solve and closed-form log-det / gradient
    n, s2, sg = 9, 0.8, 0.05
    X = np.full((n, 2), 0.37)
    kern = gp.Kern(family, 0.4, s2, sg)
    y = np.random.default_rng(4).standard_normal(n)
    np.testing.assert_allclose(gp.ky_matrix(kern, X), sg * np.eye(n) + s2 * np.ones((n, n)), rtol=1e-15)
    a_ref = (y - s2 * y.sum() / (sg + n * s2)) / sg
    np.testing.assert_allclose(gp.solve(kern, X, y), a_ref, rtol=1e-11)
    ld = (n - 1) * math.log(sg) + math.log(sg + n * s2)
    assert gp.logdet(kern, X) == pytest.approx(ld, rel=1e-12)
    g = gp.mll_grad(kern, X, y)
    assert g[0] == pytest.approx(0.0, abs=1e-12)                         # d/dl
    assert g[1] == pytest.approx(0.5 * a_ref.sum() ** 2 - 0.5 * n / (sg + n * s2), rel=1e-10)
    assert g[2] == pytest.approx(0.5 * a_ref @ a_ref - 0.5 * ((n - 1) / sg + 1 / (sg + n * s2)), rel=1e-10)


# ---------------------------------------------------------------- MLL / gradients

@pytest.mark.parametrize("family", FAMS)
def test_mll_vs_library_logpdf_and_brute(family):
    rng = np.random.default_rng(11)
    n, d = 30, 2
    X = rng.uniform(0, 1, size=(n, d))
    y = rng.standard_normal(n)
    kern = gp.Kern(family, np.array([0.3, 0.6]), 1.4, 0.05)
    ref = scipy.stats.multivariate_normal(mean=np.zeros(n), cov=gp.ky_matrix(kern, X)).logpdf(y)
    assert gp.mll(kern, X, y) == pytest.approx(ref, rel=1e-11)
    b = brute.mll(family, X.tolist(), y.tolist(), [0.3, 0.6], 1.4, 0.05)
    assert gp.mll(kern, X, y) == pytest.approx(b, rel=1e-10)


@pytest.mark.parametrize("family", FAMS)
@pytest.mark.parametrize("ard", [False, True])
def test_gradient_vs_central_fd(family, ard):
    rng = np.random.default_rng(5)
    n, d = 50, 3
    X = rng.uniform(0, 1, size=(n, d))
    y = np.sin(4 * X).sum(1) + 0.1 * rng.standard_normal(n)
    ls = rng.uniform(0.2, 0.6, size=d) if ard else 0.4
    kern = gp.Kern(family, ls, 1.3, 0.04)
    th = kern.params(d)
    g = gp.mll_grad(kern, X, y)
    fd = np.zeros_like(th)
    for p in range(len(th)):
        h = 1e-5 * th[p]
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd[p] = (gp.mll(kern.with_params(tp), X, y) - gp.mll(kern.with_params(tm), X, y)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())


def test_same_probe_estimator_exact_mode():
    # probes sqrt(N) e_c (same norm as Rademacher): the Hutchinson trace is exact
    rng = np.random.default_rng(8)
    n, d = 40, 2
    X = rng.uniform(0, 1, size=(n, d))
    y = rng.standard_normal(n)
    for fam in FAMS:
        kern = gp.Kern(fam, np.array([0.3, 0.5]), 1.1, 0.03)
        Z = math.sqrt(n) * np.eye(n)
        np.testing.assert_allclose(gp.same_probe_grad(kern, X, y, Z), gp.mll_grad(kern, X, y), rtol=1e-10)


def test_same_probe_estimator_is_unbiased():
    rng = np.random.default_rng(9)
    n = 60
    X = rng.uniform(0, 1, size=(n, 2))
    y = rng.standard_normal(n)
    kern = gp.Kern("rbf", 0.3, 1.0, 0.05)
    exact = gp.mll_grad(kern, X, y)
    draws = np.array([gp.same_probe_grad(kern, X, y, probes.rademacher(1000 + s, n, 8)) for s in range(300)])
    mean, se = draws.mean(0), draws.std(0, ddof=1) / math.sqrt(len(draws))
    assert np.all(np.abs(mean - exact) < 4 * se + 1e-12)


def test_adjoint_bilinear_matches_definition():
    rng = np.random.default_rng(12)
    n, d = 25, 2
    X = rng.uniform(0, 1, size=(n, d))
    A, B = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    w = np.array([0.5, -0.2, 1.5])
    kern = gp.Kern("matern32", np.array([0.3, 0.5]), 1.2, 0.1)
    th = kern.params(d)
    # FD of sum_c w_c A_c^T K_y(theta) B_c
    f = lambda k: float(np.sum((A * w) * (gp.ky_matrix(k, X) @ B)))
    fd = []
    for p in range(len(th)):
        h = 1e-6 * th[p]
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd.append((f(kern.with_params(tp)) - f(kern.with_params(tm))) / (2 * h))
    np.testing.assert_allclose(gp.adjoint_bilinear(kern, X, A, B, w), fd, rtol=1e-6)


# ---------------------------------------------------------------- Krylov

@pytest.mark.parametrize("family", ["rbf", "matern52"])
def test_cg_equals_cholesky(family):
    w = inputs.exact1k(n=300)
    kern = gp.Kern(family, 0.2, 1.0, 0.01)
    B = np.stack([w.y, np.random.default_rng(0).standard_normal(300)], 1)
    x, al, be, it = krylov.cg(lambda V: gp.ky_matvec(kern, w.X, V), B, tol=1e-12)
    np.testing.assert_allclose(x, gp.solve(kern, w.X, B), rtol=1e-9, atol=1e-9 * np.abs(x).max())
    assert np.all(gp.solve_residual(kern, w.X, B, x) <= 1e-11)
    # zero right-hand side: zero iterations, zero solution
    x0, _, _, it0 = krylov.cg(lambda V: gp.ky_matvec(kern, w.X, V), np.zeros(300), tol=1e-6)
    assert it0[0] == 0 and not x0.any()


def test_cg_tridiagonal_equals_lanczos():
    rng = np.random.default_rng(21)
    n = 200
    X = rng.uniform(0, 1, size=(n, 2))
    kern = gp.Kern("rbf", 0.25, 1.0, 0.05)
    A = gp.ky_matrix(kern, X)
    z = np.sign(rng.standard_normal(n))
    # short run: plain CG keeps its residuals orthogonal to working accuracy here
    m = 8
    _, al, be, _ = krylov.cg(lambda V: A @ V, z, tol=0.0, max_iter=m)
    dc, oc = krylov.cg_to_tridiag(al[0], be[0])
    dl, ol = krylov.lanczos(lambda v: A @ v, z, m)
    np.testing.assert_allclose(dc, dl, rtol=1e-8)
    np.testing.assert_allclose(np.abs(oc), np.abs(ol), rtol=1e-8)


def test_slq_converged_equals_exact_quadratic_form():
    rng = np.random.default_rng(22)
    n = 150
    X = rng.uniform(0, 1, size=(n, 2))
    kern = gp.Kern("matern52", 0.3, 1.0, 0.05)
    A = gp.ky_matrix(kern, X)
    Z = probes.rademacher(77, n, 4)
    # exact z^T log(A) z by a second library route (matrix logarithm)
    L = scipy.linalg.logm(A).real
    exact = np.einsum("ic,ij,jc->c", Z, L, Z)
    np.testing.assert_allclose(krylov.quadform_log(A, Z), exact, rtol=1e-9)
    _, q, it = krylov.slq_logdet(lambda V: A @ V, Z, tol=1e-12)
    np.testing.assert_allclose(q, exact, rtol=1e-8)
    # Lanczos run to m = n reproduces it as well
    dl, ol = krylov.lanczos(lambda v: A @ v, Z[:, 0], n)
    assert krylov.quadrature(dl, ol, float(Z[:, 0] @ Z[:, 0])) == pytest.approx(exact[0], rel=1e-8)


def test_slq_unbiased_for_logdet():
    rng = np.random.default_rng(23)
    n = 120
    X = rng.uniform(0, 1, size=(n, 2))
    kern = gp.Kern("rbf", 0.2, 1.0, 0.05)
    A = gp.ky_matrix(kern, X)
    Z = probes.rademacher(5, n, 400)
    q = krylov.quadform_log(A, Z)
    exact = float(np.linalg.slogdet(A)[1])
    assert abs(q.mean() - exact) < 4 * q.std(ddof=1) / math.sqrt(len(q))
    assert gp.logdet(kern, X) == pytest.approx(exact, rel=1e-12)


# ---------------------------------------------------------------- probes, bf16

def _golden_splitmix():
    out, seed = {}, None
    with open(os.path.join(HERE, "golden", "splitmix64.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("seed"):
                seed = int(line.split()[1])
                out[seed] = []
            else:
                out[seed].append(int(line))
    return out


def test_splitmix64_published_vectors():
    for seed, vals in _golden_splitmix().items():
        assert probes.stream(seed, len(vals)) == vals


def test_rademacher_counter_layout():
    seed, n, p = 300, 7, 3
    Z = probes.rademacher(seed, n, p)
    s = probes.stream(seed, n * p)
    for c in range(p):
        for j in range(n):
            assert Z[j, c] == (1.0 if s[c * n + j] >> 63 == 0 else -1.0)
    big = probes.rademacher(1, 4000, 8)
    assert set(np.unique(big)) == {-1.0, 1.0}
    assert abs(big.mean()) < 0.03


def test_bf16_rounding():
    one = np.float32(1.0)
    tie_even = np.float32(1.0 + 2.0 ** -8)            # halfway between 1 and 1+2^-7 -> 1
    tie_odd = np.float32(1.0 + 3 * 2.0 ** -8)         # halfway between 1+2^-7 and 1+2^-6 -> 1+2^-6
    above = np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)  # just above the tie -> 1+2^-7
    got = bf16.round_bf16(np.array([one, tie_even, tie_odd, above, -tie_odd]))
    np.testing.assert_array_equal(got, np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -(1 + 2.0 ** -6)],
                                                np.float32))
    # agree with the library conversion on random data
    a = np.random.default_rng(0).standard_normal(100000).astype(np.float32) * 10
    lib = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(bf16.round_bf16(a), lib)
    hi, lo = bf16.split_bf16(a)
    assert np.all(np.abs(a - hi - lo) <= np.abs(a) * 2.0 ** -15)


def test_bf16_three_way_split_is_exact():
    # Normal binary32 values over 52 binades: h + m + l reproduces a exactly,
    # each piece is a bfloat16 value, and the pieces shrink by >= 2^8.
    rng = np.random.default_rng(4)
    a = (rng.standard_normal(200000) * np.exp(rng.uniform(-18, 18, 200000))).astype(np.float32)
    h, m, l = bf16.split3_bf16(a)
    for x in (h, m, l):
        np.testing.assert_array_equal(bf16.round_bf16(x), x)
    np.testing.assert_array_equal(h.astype(np.float64) + m + l, a.astype(np.float64))
    assert np.all(np.abs(m) <= np.abs(h) * 2.0 ** -8)
    assert np.all(np.abs(l) <= np.abs(m) * 2.0 ** -8)
    # 1 + 2^-8 + 2^-16 + 2^-23 (24 significant bits) splits as 1 + 2^-8 + (2^-16 + 2^-23)
    v = np.float32(1.0 + 2.0 ** -9 + 2.0 ** -17 + 2.0 ** -23)
    hv, mv, lv = bf16.split3_bf16(np.array([v]))
    assert float(hv[0]) + float(mv[0]) + float(lv[0]) == float(v)


def test_bf16_x3_tile_product_is_binary32_accurate():
    # The six-product x3 model is within a few binary32 roundings of the exact
    # product; x2 is not (its pieces keep 16 bits).
    rng = np.random.default_rng(5)
    K = rng.uniform(0, 1, (64, 512)).astype(np.float32)
    V = rng.standard_normal((512, 8)).astype(np.float32)
    exact = K.astype(np.float64) @ V.astype(np.float64)
    absk = np.abs(K).astype(np.float64) @ np.abs(V).astype(np.float64)
    e3 = np.abs(bf16.tile_product_x3(K, V) - exact) / absk
    e2 = np.abs(bf16.tile_product_x2(K, V) - exact) / absk
    assert e3.max() <= 2.0 ** -26     # measured 2^-29.8 here
    assert e2.max() > 2.0 ** -24      # measured 2^-20.4 here
    # x2 keeps 16 bits of each operand: every term's error is at most
    # |k v| (2^-16 for the dropped lo*lo product + 2 * 2^-17 for rounding the
    # two lo pieces), so |e2| <= 2^-15 of sum |k||v| in the worst case; random
    # data cancels far below that
    assert e2.max() <= 2.0 ** -17
    e1 = np.abs(bf16.tile_product_x1(K, V) - exact) / absk
    assert 2.0 ** -12 < e1.max() <= 2.0 ** -7   # two RNE roundings of 2^-9 each


def _bits(rng, shape, keep):
    """float32 values with at most `keep` significant bits (exactly
    representable in that many bits), magnitudes 2^-6..2^2."""
    m = rng.integers(2 ** (keep - 1), 2 ** keep, size=shape).astype(np.float64)
    e = rng.integers(-6 - keep, 3 - keep, size=shape).astype(np.float64)
    s = rng.choice([-1.0, 1.0], size=shape)
    return (s * m * 2.0 ** e).astype(np.float32)


def test_bf16_tile_models_exact_on_short_operands():
    # Operands with <= 8 significant bits are bfloat16 values: their lo pieces
    # vanish and the models reduce to exact products.  With one operand of 8
    # bits and the other of 16, hi + lo reproduces the 16-bit operand exactly,
    # so x2 must be exact as well: each of its three products is needed (a
    # model that dropped hi*lo or lo*hi would be off by ~2^-9 here).
    rng = np.random.default_rng(17)
    K8, V8 = _bits(rng, (48, 256), 8), _bits(rng, (256, 5), 8)
    K16, V16 = _bits(rng, (48, 256), 16), _bits(rng, (256, 5), 16)
    for K, V in ((K8, V8), (K8, V16), (K16, V8)):
        exact = K.astype(np.float64) @ V.astype(np.float64)
        np.testing.assert_array_equal(bf16.tile_product_x2(K, V), exact)
        np.testing.assert_array_equal(bf16.tile_product_x3(K, V), exact)
    np.testing.assert_array_equal(bf16.tile_product_x1(K8, V8), K8.astype(np.float64) @ V8.astype(np.float64))
    # 16 x 16 bits: x2 misses exactly the lo*lo product, x3 nothing
    kh, kl = bf16.split_bf16(K16)
    vh, vl = bf16.split_bf16(V16)
    np.testing.assert_array_equal(kh.astype(np.float64) + kl, K16.astype(np.float64))
    exact = K16.astype(np.float64) @ V16.astype(np.float64)
    np.testing.assert_allclose(bf16.tile_product_x2(K16, V16) + kl.astype(np.float64) @ vl.astype(np.float64),
                               exact, rtol=0, atol=1e-15 * np.abs(exact).max())
    np.testing.assert_array_equal(bf16.tile_product_x3(K16, V16), exact)


def test_bf16_x2_bound_catches_a_dropped_cross_product():
    # A model that loses one of x2's cross products fails the x2 bound above.
    rng = np.random.default_rng(5)
    K = rng.uniform(0, 1, (64, 512)).astype(np.float32)
    V = rng.standard_normal((512, 8)).astype(np.float32)
    exact = K.astype(np.float64) @ V.astype(np.float64)
    absk = np.abs(K).astype(np.float64) @ np.abs(V).astype(np.float64)
    kh, kl = (x.astype(np.float64) for x in bf16.split_bf16(K))
    vh, vl = (x.astype(np.float64) for x in bf16.split_bf16(V))
    for wrong in (kh @ vh + kh @ vl, kh @ vh + kl @ vh):
        assert (np.abs(wrong - exact) / absk).max() > 2.0 ** -17


@pytest.mark.parametrize("family", ["rbf", "matern12", "matern32", "matern52"])
def test_kernel_matrix_f32_is_a_binary32_evaluation(family):
    # Each entry is the FP64 entry up to a few binary32 roundings: the
    # differences, squares and sum give r^2 a relative error of at most about
    # (2d + 1) u (u = 2^-24), the profile turns that into (r^2 / 2) or rho
    # times it, and the exponential and the products add a few u.
    rng = np.random.default_rng(33)
    d = 3
    X = rng.uniform(0, 1, (120, d))
    k = gp.Kern(family, np.array([0.3, 0.5, 0.2]), 1.7, 0.01)
    K = gp.kernel_matrix(k, X, X)
    K32 = gp.kernel_matrix_f32(k, X, X)
    r2 = gp.scaled_sqdist(X, X, k.ls_vec(d))
    u = 2.0 ** -24
    bound = u * (8.0 + (2 * d + 1) * (r2 + 4.0 * np.sqrt(r2)))
    rel = np.abs(K32 - K) / K
    assert np.all(rel <= bound)
    assert rel.max() > u / 4          # it is not the FP64 evaluation
    np.testing.assert_array_equal(K32, K32.T)   # the same steps for (i, j) and (j, i)
    np.testing.assert_allclose(np.diag(K32), 1.7 * np.float32(1.0), rtol=u)


def _prescaled_profile(family, q2):
    """Unit-scale kernel from q^2 = |u - u'|^2 of the prescaled coordinates, FP64."""
    if family == "rbf":
        return np.exp2(-q2)
    q = np.sqrt(q2)
    a = q * math.log(2.0)
    poly = {"matern12": 1.0, "matern32": 1.0 + a, "matern52": 1.0 + a + a * a / 3.0}[family]
    return poly * np.exp2(-q)


@pytest.mark.parametrize("family", ["rbf", "matern12", "matern32", "matern52"])
def test_kernel_matrix_f32_prescaled_form(family):
    # The prescaled form is the same kernel: with u_k = x_k c / l_k (RBF
    # c = sqrt(log2(e) / 2): 2^(-|u - u'|^2) = exp(-r^2 / 2); Matern-nu
    # c = sqrt(2 nu) log2(e): 2^(-q) = exp(-sqrt(2 nu) rho)) -- an identity
    # checked here in FP64.  In binary32 it is the exact kernel at the
    # coordinates as rounded after scaling, up to the roundings of the
    # differences, squares, sum and exponential; the rounding of each point's
    # coordinates is shared by all its entries, so the errors of a product
    # add up coherently: larger than the direct evaluation's.
    rng = np.random.default_rng(34)
    d = 2
    n = 1500
    X = rng.uniform(0, 1, (n, d))
    ls = np.array([0.05, 0.07])
    k = gp.Kern(family, ls, 1.0, 0.01)
    log2e = 1.0 / math.log(2.0)
    c = math.sqrt(log2e / 2.0) if family == "rbf" else \
        math.sqrt({"matern12": 1.0, "matern32": 3.0, "matern52": 5.0}[family]) * log2e
    rows = np.arange(0, n, 25)
    # the identity, FP64
    Ue = X * (c / ls)
    q2e = ((Ue[rows, None, :] - Ue[None, :, :]) ** 2).sum(axis=2)
    K = gp.kernel_matrix(k, X[rows], X)
    np.testing.assert_allclose(_prescaled_profile(family, q2e), K, rtol=1e-12, atol=1e-300)
    # binary32: the exact kernel at the rounded scaled coordinates
    s32 = (c / ls).astype(np.float32)
    U32 = (X.astype(np.float32) * s32).astype(np.float64)
    q2 = ((U32[rows, None, :] - U32[None, :, :]) ** 2).sum(axis=2)
    ref = _prescaled_profile(family, q2)
    K32p = gp.kernel_matrix_f32(k, X[rows], X, prescaled=True)
    keep = ref > 1e-6
    u = 2.0 ** -24
    bound = u * (8.0 + 8.0 * (q2 + np.sqrt(q2)))
    rel = np.abs(K32p - ref)[keep] / ref[keep]
    assert np.all(rel <= bound[keep])
    # coherent errors: the product error exceeds the direct evaluation's
    # (1.3-1.6x here with ~10 neighbours per row; about 6x at 5e5 points on
    # [0, 1]^2 with l = 0.05, where each row has thousands)
    K32d = gp.kernel_matrix_f32(k, X[rows], X)
    x = rng.choice([-1.0, 1.0], n) * 100.0
    ep = np.linalg.norm((K32p - K) @ x)
    ed = np.linalg.norm((K32d - K) @ x)
    assert ep > ed, (ep, ed)
