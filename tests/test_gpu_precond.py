"""Pivoted-Cholesky preconditioner and the preconditioned solver against the
FP64 oracle (oracle/precond.py).

Pivot indices are integer decisions taken from FP32 kernel entries on the GPU
and FP64 entries in the oracle; the inputs are generic random points whose
greedy gaps are far above that rounding, so the pivots must agree exactly and
the factor columns to FP32 accuracy.  Everything downstream is compared with
the oracle evaluated on the GPU's own factor (as FP64), so that the check of
the Woodbury apply, the probes, the solver and the estimators does not depend
on the factor's rounding.
"""

import numpy as np
import pytest

from oracle import gp, krylov, precond
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, col_rel_err, dev, host, mkern, okern

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


@pytest.mark.parametrize("family", ["rbf", "matern12", "matern52"])
def test_pivoted_cholesky_matches_oracle(mf, family):
    banner(f"pivoted Cholesky rank 24, n=700 d=2 {family}")
    w = inputs.random_problem(501, 700, 2, family, ard=True, noise=0.02)
    L, piv = mf.pivoted_cholesky(mkern(w), dev(w.X), 24)
    Lo, pivo = precond.pivoted_cholesky(okern(w), w.X, 24)
    np.testing.assert_array_equal(host(piv), pivo)
    assert np.abs(host(L).T - Lo).max() <= 2e-5 * np.sqrt(w.outputscale)


def test_pivoted_cholesky_ragged_and_rank_floor(mf):
    banner("pivoted Cholesky: n=257 rank 40; identical points give zero columns past rank 1")
    w = inputs.random_problem(502, 257, 3, "rbf", ard=False, noise=0.02)
    L, piv = mf.pivoted_cholesky(mkern(w), dev(w.X), 40)
    Lo, pivo = precond.pivoted_cholesky(okern(w), w.X, 40)
    np.testing.assert_array_equal(host(piv), pivo)
    assert np.abs(host(L).T - Lo).max() <= 2e-5 * np.sqrt(w.outputscale)
    Xs = np.full((50, 2), 0.3, np.float32)
    k = mf.Kernel("rbf", 0.5, 1.7, 0.1)
    L, piv = mf.pivoted_cholesky(k, dev(Xs), 5)
    Lh = host(L)
    np.testing.assert_allclose(Lh[0], np.sqrt(1.7), rtol=1e-6)
    assert np.all(Lh[1:] == 0.0)


@pytest.mark.parametrize("rank", [0, 1, 17, 64])
def test_precond_apply_probes_and_logdet(mf, rank):
    banner(f"Woodbury apply and probes, rank {rank}, n=1537 (ragged split), t=9")
    w = inputs.random_problem(503, 1537, 3, "matern32", ard=True, noise=0.03)
    if rank:
        L, _ = mf.pivoted_cholesky(mkern(w), dev(w.X), rank)
    else:
        L = dev(np.zeros((0, 1537), np.float32))
    L64 = host(L).T.astype(np.float64)
    s2n = float(np.float32(w.noise))     # the library holds sigma^2 in binary32
    R = inputs.gaussian_rhs(7, 1537, 9)
    Z, ld = mf.precond_apply(L, w.noise, dev(R))
    ref = precond.precond_solve(L64, s2n, R.astype(np.float64))
    assert col_rel_err(host(Z), ref).max() <= 1e-5
    assert ld == pytest.approx(precond.precond_logdet(L64, s2n, 1537), rel=1e-10)
    E = inputs.gaussian_rhs(8, max(rank, 1), 5)[:rank] if rank else np.zeros((0, 5), np.float32)
    G = inputs.gaussian_rhs(9, 1537, 5)
    Zp = mf.precond_probes(L, w.noise, dev(np.ascontiguousarray(E)), dev(G))
    np.testing.assert_allclose(host(Zp), precond.precond_probes(L64, s2n, E, G), rtol=1e-5, atol=1e-5)


def test_pcg_solves_with_fewer_iterations(mf):
    banner("preconditioned CG exact1k [y, 8 probes], rank 60 vs plain CG")
    w = inputs.exact1k(probes=8)
    B = np.concatenate([w.y[:, None], w.Z], axis=1)
    L, _ = mf.pivoted_cholesky(mkern(w), dev(w.X), 60)
    x, info, _, st = mf.precond_cg_solve(mkern(w), dev(w.X), dev(B), L, tol=1e-6)
    assert st == mf.OK, info
    assert max(i["rel_resid_true"] for i in info) <= 1e-6
    assert col_rel_err(host(x), gp.solve(okern(w), w.X, B)).max() <= 1e-4
    _, pinfo, _, _ = mf.cg_solve(mkern(w), dev(w.X), dev(B), tol=1e-6)
    it_p = max(i["iters"] for i in info)
    it_c = max(i["iters"] for i in pinfo)
    print(f"iterations: preconditioned {it_p}, plain {it_c}")
    assert it_p < it_c


def test_pcg_tridiagonal_matches_oracle(mf):
    banner("PCG first-cycle coefficients vs oracle PCG on the GPU's factor")
    w = inputs.random_problem(504, 900, 2, "rbf", ard=True, noise=0.05)
    L, _ = mf.pivoted_cholesky(mkern(w), dev(w.X), 20)
    L64 = host(L).T.astype(np.float64)
    b = w.y[:, None].astype(np.float32)
    _, info, lan, st = mf.precond_cg_solve(mkern(w), dev(w.X), dev(b), L, tol=1e-6, want_lanczos=True)
    assert st == mf.OK
    A = gp.ky_matrix(okern(w), w.X)
    _, al, be, _, _ = precond.pcg(lambda V: A @ V, L64, w.noise, b.astype(np.float64), tol=1e-12, max_iter=8)
    # the FP32-entry operator and the FP64 one separate as the Krylov space
    # grows (the eighth off-diagonal already differs by 1%): compare six steps
    got = host(lan)[0, :6]
    d1, o1 = krylov.cg_to_tridiag(got[:, 0], got[:, 1])
    d2, o2 = krylov.cg_to_tridiag(al[0][:6], be[0][:6])
    np.testing.assert_allclose(d1, d2, rtol=1e-4)
    np.testing.assert_allclose(o1, o2, rtol=1e-3)


def test_precond_mll_same_probe(mf):
    banner("preconditioned mll + grad exact1k p=16 rank 40 vs same-probe oracle")
    w = inputs.exact1k()
    k = okern(w)
    L, _ = mf.pivoted_cholesky(mkern(w), dev(w.X), 40)
    L64 = host(L).T.astype(np.float64)
    E = inputs.gaussian_rhs(11, 40, 16)
    G = inputs.gaussian_rhs(12, w.n, 16)
    Z = mf.precond_probes(L, w.noise, dev(E), dev(G))
    r = mf.precond_mll_and_grad(mkern(w), dev(w.X), dev(w.y), Z, L, tol=1e-6)
    assert r["status"] == mf.OK
    Z64 = host(Z).astype(np.float64)
    ld = precond.same_probe_logdet(k, w.X, L64, Z64)
    assert r["logdet"] == pytest.approx(ld, rel=1e-4)
    g = precond.same_probe_grad(k, w.X, w.y, Z64, L64)
    assert np.linalg.norm(np.array(r["grad"]) - g) / np.linalg.norm(g) <= 1e-3
    mll = -0.5 * (float(w.y.astype(np.float64) @ gp.solve(k, w.X, w.y)) + ld + w.n * np.log(2 * np.pi))
    assert r["mll"] == pytest.approx(mll, rel=1e-4)


def test_precond_exact_mode_vs_exact_values(mf):
    # z_c = sqrt(n) P^{1/2} e_c makes both estimators exact: log-det and gradient
    # must equal the Cholesky values.
    banner("preconditioned mll exact mode n=64 rank 10 vs exact log-det and gradient")
    w = inputs.random_problem(505, 64, 3, "rbf", ard=True, noise=0.05)
    k = okern(w)
    L, _ = mf.pivoted_cholesky(mkern(w), dev(w.X), 10)
    L64 = host(L).T.astype(np.float64)
    P = L64 @ L64.T + w.noise * np.eye(64)
    ev, Q = np.linalg.eigh(P)
    Z = (np.sqrt(64) * (Q * np.sqrt(ev)) @ Q.T).astype(np.float32)
    r = mf.precond_mll_and_grad(mkern(w), dev(w.X), dev(w.y), dev(Z), L, tol=1e-7)
    assert r["status"] == mf.OK
    assert r["logdet"] == pytest.approx(gp.logdet(k, w.X), rel=1e-4, abs=1e-3)
    g = gp.mll_grad(k, w.X.astype(np.float64), w.y.astype(np.float64))
    assert np.linalg.norm(np.array(r["grad"]) - g) / np.linalg.norm(g) <= 1e-3


def test_pcg_full_rbf100k(mf):
    banner("preconditioned CG rbf100k [y, 32 probes], rank 256")
    w = inputs.rbf100k()
    B = np.concatenate([w.y[:, None], w.Z], axis=1)
    L, _ = mf.pivoted_cholesky(mkern(w), dev(w.X), 256)
    x, info, _, st = mf.precond_cg_solve(mkern(w), dev(w.X), dev(B), L, tol=1e-6,
                                         progress=lambda it, rr: print(f"pcg {it} {rr:.2e}", flush=True))
    assert st == mf.OK, info
    assert max(i["rel_resid_true"] for i in info) <= 1e-6
    it = max(i["iters"] for i in info)
    print(f"rbf100k preconditioned iterations: {it}")
    # FP64-entry residual of the solution of the FP32-entry operator on sampled
    # rows: the returned 1e-6 plus the part FP32 entries leave, computed by the
    # oracle for this solution (the probe columns carry the larger one, since
    # |K^-1 z| ~ |z| / sigma^2); factor 2 for the different rounding of the
    # oracle's binary32 evaluation
    rows = np.random.default_rng(3).choice(w.n, size=256, replace=False)
    res = gp.solve_residual(okern(w), w.X, B, host(x), rows=rows)
    floor = gp.fp32_entry_floor(okern(w), w.X, B, host(x), rows)
    print(f"sampled FP64 residuals up to {res.max():.2e}, FP32-entry floors up to {floor.max():.2e}")
    assert np.all(res <= 2 * floor + 2e-6), (res, floor)


def test_pcg_rbf500k_sampled_residual(mf):
    # The 500k workload (N = 5e5, d = 2, l = 0.05, [y, 16 probes]) with the
    # rank-1024 preconditioner: every column to 1e-6, and the oracle's FP64
    # residual of the returned solution on 1024 sampled rows within the
    # returned 1e-6 plus its computed FP32-entry floor.
    banner("preconditioned CG rbf500k [y, 16 probes], rank 1024, sampled FP64 residual")
    w = inputs.rbf500k()
    B = np.concatenate([w.y[:, None], w.Z], axis=1)
    L, _ = mf.pivoted_cholesky(mkern(w), dev(w.X), 1024)
    x, info, _, st = mf.precond_cg_solve(mkern(w), dev(w.X), dev(B), L, tol=1e-6)
    assert st == mf.OK, info
    assert max(i["rel_resid_true"] for i in info) <= 1e-6
    print(f"rbf500k preconditioned iterations: {max(i['iters'] for i in info)}")
    rows = np.random.default_rng(5).choice(w.n, size=1024, replace=False)
    xs = host(x)
    res = gp.solve_residual(okern(w), w.X, B, xs, rows=rows)
    floor = gp.fp32_entry_floor(okern(w), w.X, B, xs, rows)
    print(f"sampled FP64 residuals up to {res.max():.2e}, FP32-entry floors up to {floor.max():.2e}")
    assert np.all(res <= 2 * floor + 2e-6), (res, floor)
