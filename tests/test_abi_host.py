"""Host-side checks of the C-ABI library: it loads, exports what include/mfgp.h
declares, validates arguments before any launch, sizes workspaces, and its
host-only stochastic-Lanczos quadrature matches the oracle.  No GPU needed."""

import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle import gp, krylov, probes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfgp.h")
LIB_PATH = os.path.join(ROOT, "paper_2605_17898_amd", "libmfgp.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB_PATH), reason="libmfgp.so not built")


@pytest.fixture(scope="module")
def m():
    from paper_2605_17898_amd import mfgp
    return mfgp


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfgp_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = C.CDLL(LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings_and_version(m):
    assert m.LIB.mfgp_version() >= 100
    for code in range(7):
        assert m.LIB.mfgp_status_string(code)
    assert m.LIB.mfgp_status_string(99) == b"unknown status"


def test_num_params(m):
    assert m.Kernel("rbf", 0.3).n_params(4) == 3
    assert m.Kernel("matern52", [0.3, 0.2, 0.5]).n_params(3) == 5


def test_periodic_params_and_feature_dim(m):
    # [l.., p, s2, sigma^2]; the size queries take the 2 d circle features
    assert m.Kernel("periodic", 0.3, period=0.5).n_params(2) == 4
    assert m.Kernel("periodic", [0.3, 0.2, 0.5], period=0.5).n_params(3) == 6
    assert m.Kernel("periodic", 0.3).feature_dim(3) == 6
    assert m.Kernel("matern32", 0.3).feature_dim(3) == 3
    assert m.LIB.mfgp_feature_dim(None) == 0


@pytest.mark.parametrize("period,d,want", [
    (0.0, 2, 1), (-1.0, 2, 1), (float("nan"), 2, 1), (float("inf"), 2, 1),
    (0.5, 5, 6),     # 10 features > MFGP_MAX_D
    (0.5, 4, 3),     # valid: stops at the workspace check
])
def test_periodic_kernel_checks_before_launch(m, period, d, want):
    k = m.Kernel("periodic", 0.3, 1.0, 0.01, period=period).struct(d)
    dummy = C.c_void_p(16)
    st = m.LIB.mfgp_kernel_matvec(C.byref(k), dummy, 10, dummy, 1, C.c_void_p(32), 0, dummy, 16, None)
    assert st == want


def test_sum_and_linear_params_and_checks(m):
    rbf, per, lin = m.Kernel("rbf", [0.4, 0.9], 1.1, 0.04), m.Kernel("periodic", 0.7, 0.6, period=0.45), \
        m.Kernel("linear", 1.0, 0.3)
    assert lin.n_params(2) == 2 and lin.feature_dim(2) == 2
    ksum = rbf + per + lin
    assert ksum.n_params(2) == 8          # [l1, l2, s2 | l, p, s2 | s2 | sigma^2]
    assert ksum.feature_dim(2) == 8
    dummy = C.c_void_p(16)
    L = m.LIB

    def matvec(k, d=2, ws=16):
        return L.mfgp_kernel_matvec(C.byref(k), dummy, 10, dummy, 1, C.c_void_p(32), 0, dummy, ws, None)

    assert matvec(ksum.struct(2)) == m.ERR_WORKSPACE     # valid chain: stops at the size check
    five = rbf + rbf + rbf + rbf + rbf
    assert matvec(five.struct(2)) == m.UNSUPPORTED        # more than MFGP_MAX_TERMS
    bad = ksum.struct(2)
    bad._chain_ref[0][1].d = 3                             # terms must share d
    assert matvec(bad) == m.ERR_ARG
    neg = (rbf + m.Kernel("linear", 1.0, -0.3)).struct(2)
    assert matvec(neg) == m.ERR_ARG
    # the preconditioned calls take one stationary or periodic term
    for k in (ksum.struct(2), lin.struct(2)):
        assert L.mfgp_pivoted_cholesky(C.byref(k), dummy, 10, 2, dummy, dummy, dummy, 1 << 20, None) == m.UNSUPPORTED
    # feature dimensions above MFGP_MAX_D are valid for sums in the size queries
    assert m.workspace_bytes(m.OP_CG, 1000, 12, 3) > 0
    assert m.workspace_bytes(m.OP_CG, 1000, 33, 3) == 0


def test_product_params_and_checks(m):
    rbf, per, lin = m.Kernel("rbf", [0.6, 1.4], 1.3, 0.05), m.Kernel("periodic", 0.8, period=0.45), \
        m.Kernel("linear", 1.0, 0.3)
    prod = rbf * per
    assert prod.n_params(2) == 6          # [l1, l2 | l, p | s2 | sigma^2]
    assert prod.feature_dim(2) == 6
    assert (prod + lin).n_params(2) == 7
    assert (m.Kernel("rbf", 0.5) * m.Kernel("rbf", 0.7)).feature_dim(4) == 8
    dummy = C.c_void_p(16)
    L = m.LIB

    def matvec(k, ws=16):
        return L.mfgp_kernel_matvec(C.byref(k), dummy, 10, dummy, 1, C.c_void_p(32), 0, dummy, ws, None)

    assert matvec(prod.struct(2)) == m.ERR_WORKSPACE
    assert matvec((prod + lin).struct(2)) == m.ERR_WORKSPACE
    assert matvec((per * per).struct(1)) == m.UNSUPPORTED                 # two periodic factors
    # products with Matern or Linear factors: valid (the general product);
    # parameters: each factor's lengthscales (none for Linear), then s2, sigma^2
    gm = rbf * m.Kernel("matern32", 0.5)
    gl = rbf * lin
    assert matvec(gm.struct(2)) == m.ERR_WORKSPACE
    assert matvec(gl.struct(2)) == m.ERR_WORKSPACE
    assert gm.n_params(2) == 5 and gm.feature_dim(2) == 4
    assert gl.n_params(2) == 4 and gl.feature_dim(2) == 4
    # ... but not in the bf16 forms, nor for the preconditioner
    assert L.mfgp_kernel_matvec(C.byref(gm.struct(2)), dummy, 10, dummy, 1, C.c_void_p(32), m.PRECISIONS["bf16x2"],
                                dummy, 16, None) == m.UNSUPPORTED
    assert L.mfgp_pivoted_cholesky(C.byref(gm.struct(2)), dummy, 10, 2, dummy, dummy, dummy, 16, None) \
        == m.UNSUPPORTED
    big = m.Kernel("rbf", 0.5, 1.0, 0.1) * m.Kernel("periodic", 0.5, period=1.0)
    assert matvec(big.struct(3)) == m.UNSUPPORTED                          # 9 features > MFGP_MAX_D
    bad = (rbf * m.Kernel("periodic", 0.8, period=-1.0)).struct(2)
    assert matvec(bad) == m.ERR_ARG
    # a product term alone is valid for the preconditioner
    assert L.mfgp_pivoted_cholesky(C.byref(prod.struct(2)), dummy, 10, 2, dummy, dummy, dummy, 16, None) \
        == m.ERR_WORKSPACE


def test_ski_checks_before_launch(m):
    dummy = C.c_void_p(16)
    L = m.LIB
    g = m.ski_grid([64, 32])

    def matvec(k, grid, d=2, ws=16):
        return L.mfgp_ski_matvec(C.byref(k.struct(d)), dummy, 10, C.byref(grid), dummy, 1, C.c_void_p(32), dummy,
                                 ws, None)

    rbf = m.Kernel("rbf", 0.3, 1.0, 0.1)
    assert matvec(rbf, g) == m.ERR_WORKSPACE
    assert matvec(m.Kernel("periodic", 0.3, period=0.5), g) == m.ERR_WORKSPACE
    assert matvec(rbf + rbf, g) == m.UNSUPPORTED
    assert matvec(m.Kernel("linear", 1.0), g) == m.UNSUPPORTED
    assert matvec(rbf, m.ski_grid([64, 32, 8]), d=4) == m.UNSUPPORTED          # d > 3
    assert matvec(rbf, m.ski_grid([64, 4])) == m.ERR_ARG                        # m_k < 5
    assert matvec(rbf, m.ski_grid([64, 32], lo=[0.0, 1.0], hi=[1.0, 0.5])) == m.ERR_ARG   # hi < lo
    assert matvec(rbf, m.ski_grid([40000, 40000])) == m.UNSUPPORTED             # 2^31 embedded nodes
    assert L.mfgp_ski_matvec(C.byref(rbf.struct(2)), dummy, 10, None, dummy, 1, C.c_void_p(32), dummy, 16,
                             None) == m.ERR_ARG
    a = L.mfgp_ski_workspace_bytes(m.OP_CG, 10000, 1, 3, C.byref(m.ski_grid([1000])))
    b = L.mfgp_ski_workspace_bytes(m.OP_CG, 100000, 1, 3, C.byref(m.ski_grid([1000])))
    assert 0 < a < b < 11 * a
    assert L.mfgp_ski_workspace_bytes(m.OP_ADJOINT, 100, 1, 3, C.byref(m.ski_grid([100]))) == 0
    assert L.mfgp_ski_workspace_bytes(m.OP_MLL, 100, 1, 9, C.byref(m.ski_grid([100]))) > 0
    assert L.mfgp_ski_workspace_bytes(m.OP_MLL, 100, 1, 1, C.byref(m.ski_grid([100]))) == 0


def test_workspace_sizes(m):
    for op in range(6):
        t = 2 if op != m.OP_PREDICT else 3
        mi = 100 if op == m.OP_PREDICT else 0
        assert m.workspace_bytes(op, 1000, 3, t, 0, mi) > 0
    assert m.workspace_bytes(m.OP_MATVEC, 0, 3, 1) == 0
    assert m.workspace_bytes(m.OP_MATVEC, 10, 33, 1) == 0     # d > MFGP_MAX_TERMS * MFGP_MAX_D
    assert m.workspace_bytes(m.OP_MATVEC, 10, 2, 0) == 0
    assert m.workspace_bytes(m.OP_MLL, 10, 2, 1) == 0         # needs >= 1 probe
    # O(n) workspace: 10x the points -> about 10x the bytes
    a = m.workspace_bytes(m.OP_CG, 10000, 4, 33)
    b = m.workspace_bytes(m.OP_CG, 100000, 4, 33)
    assert b < 12 * a


def _kern(m, **kw):
    k = m.Kernel("rbf", 0.3, 1.0, 0.01).struct(2)
    for key, v in kw.items():
        setattr(k, key, v)
    return k


@pytest.mark.parametrize("field,value,want", [
    ("family", 7, 1), ("d", 0, 1), ("d", 9, 6), ("outputscale", 0.0, 1),
    ("outputscale", float("nan"), 1), ("noise", -1.0, 1),
])
def test_matvec_rejects_bad_kernel_before_launch(m, field, value, want):
    k = _kern(m, **{field: value})
    dummy = C.c_void_p(16)
    st = m.LIB.mfgp_kernel_matvec(C.byref(k), dummy, 10, dummy, 1, C.c_void_p(32), 0, dummy, 1 << 20, None)
    assert st == want


def test_matvec_argument_checks(m):
    k = _kern(m)
    d = C.c_void_p(16)
    L = m.LIB
    assert L.mfgp_kernel_matvec(None, d, 10, d, 1, C.c_void_p(32), 0, d, 1 << 20, None) == m.ERR_ARG
    assert L.mfgp_kernel_matvec(C.byref(k), None, 10, d, 1, C.c_void_p(32), 0, d, 1 << 20, None) == m.ERR_ARG
    assert L.mfgp_kernel_matvec(C.byref(k), d, 0, d, 1, C.c_void_p(32), 0, d, 1 << 20, None) == m.ERR_ARG
    assert L.mfgp_kernel_matvec(C.byref(k), d, 10, d, 0, C.c_void_p(32), 0, d, 1 << 20, None) == m.ERR_ARG
    assert L.mfgp_kernel_matvec(C.byref(k), d, 10, d, 1, d, 0, d, 1 << 20, None) == m.ERR_ARG   # KV aliases V
    assert L.mfgp_kernel_matvec(C.byref(k), d, 10, d, 1, C.c_void_p(32), 7, d, 1 << 20, None) == m.ERR_ARG   # no precision 7
    assert L.mfgp_kernel_matvec(C.byref(k), d, 10, d, 1, C.c_void_p(32), 0, d, 16, None) == m.ERR_WORKSPACE


def test_cg_and_mll_argument_checks(m):
    k = _kern(m)
    d = C.c_void_p(16)
    L = m.LIB
    info = (m.CgInfoT * 2)()
    o = m.cg_opts(tol=0.0)
    assert L.mfgp_cg_solve(C.byref(k), d, 10, d, 1, d, C.byref(o), info, None, d, 1 << 30, None) == m.ERR_ARG
    o = m.cg_opts(tol=1e-6)
    k0 = _kern(m, noise=0.0)   # a solve needs sigma^2 > 0
    assert L.mfgp_cg_solve(C.byref(k0), d, 10, d, 1, d, C.byref(o), info, None, d, 1 << 30, None) == m.ERR_ARG
    assert L.mfgp_cg_solve(C.byref(k), d, 10, d, 1, d, C.byref(o), info, None, d, 64, None) == m.ERR_WORKSPACE
    mll = C.c_double()
    assert L.mfgp_mll_and_grad(C.byref(k), d, 10, d, 0, None, C.byref(o), C.byref(mll), None, None, None,
                               None, d, 1 << 30, None) == m.ERR_ARG
    assert L.mfgp_rademacher(1, 0, 3, d, None) == m.ERR_ARG
    assert L.mfgp_slq_quadrature(None, 3, 1.0, C.byref(mll)) == m.ERR_ARG


@pytest.mark.parametrize("family", ["rbf", "matern32"])
def test_host_slq_matches_oracle_quadrature(m, family):
    rng = np.random.default_rng(4)
    n = 200
    X = rng.uniform(0, 1, size=(n, 2))
    kern = gp.Kern(family, 0.25, 1.0, 0.03)
    A = gp.ky_matrix(kern, X)
    Z = probes.rademacher(91, n, 3)
    _, al, be, it = krylov.cg(lambda V: A @ V, Z, tol=1e-10)
    exact = krylov.quadform_log(A, Z)
    for c in range(3):
        coeffs = list(zip(al[c], be[c]))
        q_lib = m.slq_quadrature(coeffs, n)
        q_orc = krylov.quadrature(*krylov.cg_to_tridiag(al[c], be[c]), n)
        assert q_lib == pytest.approx(q_orc, rel=1e-11)
        assert q_lib == pytest.approx(exact[c], rel=1e-7)


def test_host_slq_special_cases(m):
    # one step: T = [1/alpha], q = |z|^2 log(1/alpha)
    assert m.slq_quadrature([(0.5, 0.0)], 4.0) == pytest.approx(4.0 * math.log(2.0), rel=1e-15)
    # a breakdown coefficient is reported, not hidden
    with pytest.raises(m.MfgpError):
        m.slq_quadrature([(-1.0, 0.1), (1.0, 0.1)], 4.0)
    # random SPD tridiagonal against a dense eigen-solve
    rng = np.random.default_rng(3)
    for mlen in (2, 7, 60, 300):
        al = rng.uniform(0.1, 2.0, size=mlen)
        be = rng.uniform(0.0, 0.9, size=mlen)
        dg, of = krylov.cg_to_tridiag(al, be)
        T = np.diag(dg) + np.diag(of, 1) + np.diag(of, -1)
        w, Q = np.linalg.eigh(T)
        if w.min() <= 0:
            continue
        ref = 3.0 * float(np.sum(Q[0] ** 2 * np.log(w)))
        assert m.slq_quadrature(list(zip(al, be)), 3.0) == pytest.approx(ref, rel=1e-10, abs=1e-12)


def test_host_slq_scale_covariance(m):
    # CG coefficients alpha / c, beta belong to c T, and e_1^T log(c T) e_1 =
    # log c + e_1^T log(T) e_1: the quadrature must follow at magnitudes where
    # squaring the tridiagonal's entries would overflow or underflow
    rng = np.random.default_rng(5)
    al = rng.uniform(0.1, 2.0, size=80)
    be = rng.uniform(0.0, 0.9, size=80)
    base = m.slq_quadrature(list(zip(al, be)), 3.0)
    for c in (2.0 ** 600, 1e150, 2.0 ** -600, 1e-170):
        q = m.slq_quadrature(list(zip(al / c, be)), 3.0)
        assert q == pytest.approx(base + 3.0 * math.log(c), rel=1e-12, abs=1e-9)


def test_struct_layouts_match_the_header(m, tmp_path):
    # Compile a C probe against include/mfgp.h and compare sizes and offsets
    # with the ctypes mirrors the binding passes across the ABI.
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "probe.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "mfgp.h"\n'
        'int main(void) {\n'
        '  printf("%zu %zu %zu %zu\\n", sizeof(mfgp_kernel), sizeof(mfgp_cg_opts), sizeof(mfgp_cg_info),'
        ' sizeof(mfgp_batch));\n'
        '  printf("%zu %zu %zu\\n", offsetof(mfgp_cg_opts, probe_seed), offsetof(mfgp_cg_opts, progress),'
        ' offsetof(mfgp_cg_info, replacements));\n'
        '  return 0;\n}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(v) for v in out]
    assert sizes[:4] == [C.sizeof(m.KernelT), C.sizeof(m.CgOptsT), C.sizeof(m.CgInfoT), C.sizeof(m.BatchT)]
    assert sizes[4] == m.CgOptsT.probe_seed.offset
    assert sizes[5] == m.CgOptsT.progress.offset
    assert sizes[6] == m.CgInfoT.replacements.offset


def test_variance_argument_checks(m):
    # every rejection happens on the host, before any launch
    k = _kern(m)
    d = C.c_void_p(16)
    L = m.LIB
    o = m.cg_opts(1e-6, 0, 0, -1, "fp32", False)
    nb = L.mfgp_variance_workspace_bytes(100, 2, 10, 4, 0)
    assert nb > 0
    assert L.mfgp_variance_workspace_bytes(100, 2, 0, 4, 0) == 0
    assert L.mfgp_variance_workspace_bytes(100, 2, 10, 0, 0) == 0
    assert L.mfgp_variance_workspace_bytes(100, 2, 10, 4, 7) == 0
    # O(n + m) workspace: 10x the training points -> about 10x the bytes
    assert L.mfgp_variance_workspace_bytes(100000, 2, 10, 4, 0) < 12 * L.mfgp_variance_workspace_bytes(10000, 2, 10, 4, 0)
    args = lambda **kw: dict(dict(kern=C.byref(k), X=d, n=100, Xs=d, m=10, p=4, Z=None, opts=C.byref(o),
                                  var=d, info=None, ws=d, wsb=nb, s=None), **kw)
    call = lambda a: L.mfgp_predict_variance(a["kern"], a["X"], a["n"], a["Xs"], a["m"], a["p"], a["Z"],
                                             a["opts"], a["var"], a["info"], a["ws"], a["wsb"], a["s"])
    assert call(args(kern=None)) == m.ERR_ARG
    assert call(args(X=None)) == m.ERR_ARG
    assert call(args(Xs=None)) == m.ERR_ARG
    assert call(args(var=None)) == m.ERR_ARG
    assert call(args(n=0)) == m.ERR_ARG
    assert call(args(m=0)) == m.ERR_ARG
    assert call(args(p=0)) == m.ERR_ARG
    assert call(args(opts=None)) == m.ERR_ARG
    assert call(args(wsb=16)) == m.ERR_WORKSPACE
    bad = m.cg_opts(1e-6, 0, 0, -1, "fp32", False)
    bad.tol = -1.0
    assert call(args(opts=C.byref(bad))) == m.ERR_ARG
