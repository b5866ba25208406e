"""Thin ctypes binding of libmfgp.so (C ABI in include/mfgp.h).

Argument marshalling only: every step of the path runs in the HIP library.
Tensors are caller-owned torch tensors on the GPU (float32 / float64,
contiguous); the library runs on torch's current stream.  If the library is
not built this module raises at import time: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfgp.so")

MAX_D = 8
FAMILIES = {"rbf": 0, "matern12": 1, "matern32": 2, "matern52": 3, "periodic": 4, "linear": 5}
MAX_TERMS = 4
PRECISIONS = {"fp32": 0, "bf16x1": 1, "bf16x2": 2, "fp32_valu": 3, "bf16x3": 4, "fp32_direct": 5,
              "fp32_gram": 6}
PRECISION_NAMES = {v: k for k, v in PRECISIONS.items()}
OK, ERR_ARG, ERR_HIP, ERR_WORKSPACE, NOT_CONVERGED, BREAKDOWN, UNSUPPORTED = range(7)
OP_MATVEC, OP_CG, OP_PREDICT, OP_MLL, OP_ADJOINT, OP_RESIDUAL = range(6)
OP_PCHOL, OP_PAPPLY, OP_PCG, OP_PMLL = range(6, 10)


class KernelT(C.Structure):
    pass


KernelT._fields_ = [("family", C.c_int32), ("d", C.c_int32), ("ard", C.c_int32),
                    ("lengthscale", C.c_float * MAX_D), ("outputscale", C.c_float), ("noise", C.c_float),
                    ("period", C.c_float), ("next", C.POINTER(KernelT)), ("times", C.POINTER(KernelT))]


PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_double)


class CgOptsT(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("max_refine", C.c_int32), ("precision", C.c_int32), ("warm_start", C.c_int32),
                ("no_replacement", C.c_int32), ("probe_seed", C.c_uint64), ("progress", PROGRESS_FN),
                ("progress_user", C.c_void_p), ("progress_every", C.c_int32), ("no_graph", C.c_int32)]


class CgInfoT(C.Structure):
    _fields_ = [("iters", C.c_int32), ("lanczos_len", C.c_int32), ("refinements", C.c_int32),
                ("status", C.c_int32), ("rel_resid_recurrence", C.c_double),
                ("rel_resid_true", C.c_double), ("replacements", C.c_int32),
                ("drift_skips", C.c_int32), ("stalls", C.c_int32), ("precision", C.c_int32)]


class BatchT(C.Structure):
    _fields_ = [("nprob", C.c_int32), ("pad_", C.c_int32), ("n", C.POINTER(C.c_int64)),
                ("row_off", C.POINTER(C.c_int64)), ("x_off", C.POINTER(C.c_int64)),
                ("kern", C.POINTER(KernelT))]


class SkiGridT(C.Structure):
    _fields_ = [("m", C.c_int32 * 3), ("explicit_range", C.c_int32), ("lo", C.c_float * 3), ("hi", C.c_float * 3)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(
            f"mfgp HIP library not found at {path}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (no CPU fallback exists)")
    lib = C.CDLL(path)
    P, I32, I64, SZ, D = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    KP, OP_, IP = C.POINTER(KernelT), C.POINTER(CgOptsT), C.POINTER(CgInfoT)
    sig = {
        "mfgp_workspace_bytes": (SZ, [I32, I64, I32, I32, I32, I32]),
        "mfgp_kernel_matvec": (C.c_int, [KP, P, I64, P, I32, P, I32, P, SZ, P]),
        "mfgp_kernel_matvec_noalloc": (C.c_int, [KP, P, I64, P, I32, P, I32, P]),
        "mfgp_residual": (C.c_int, [KP, P, I64, P, P, I32, P, P, P, SZ, P]),
        "mfgp_cg_solve": (C.c_int, [KP, P, I64, P, I32, P, OP_, IP, P, P, SZ, P]),
        "mfgp_predict_mean": (C.c_int, [KP, P, I64, P, I64, P, I32, P, P, SZ, P]),
        "mfgp_variance_workspace_bytes": (SZ, [I64, I32, I64, I32, I32]),
        "mfgp_predict_variance": (C.c_int, [KP, P, I64, P, I64, I32, P, OP_, P, IP, P, SZ, P]),
        "mfgp_slq_quadrature": (C.c_int, [P, I32, D, P]),
        "mfgp_mll_and_grad": (C.c_int, [KP, P, I64, P, I32, P, OP_, P, P, P, P, IP, P, SZ, P]),
        "mfgp_kernel_adjoint": (C.c_int, [KP, P, I64, P, P, I32, P, P, P, SZ, P]),
        "mfgp_rademacher": (C.c_int, [C.c_uint64, I64, I32, P, P]),
        "mfgp_num_params": (C.c_int, [KP]),
        "mfgp_feature_dim": (C.c_int, [KP]),
        "mfgp_timing_enable": (C.c_int, [I32]),
        "mfgp_timing_read": (C.c_int, [I32, P, P, P, P]),
        "mfgp_timing_phases": (C.c_int, [P, P, P]),
        "mfgp_batch_plan_create": (C.c_int, [C.POINTER(BatchT), I32, I32, I32, I32, C.POINTER(P)]),
        "mfgp_batch_plan_destroy": (C.c_int, [P]),
        "mfgp_batch_workspace_bytes": (SZ, [P]),
        "mfgp_batch_plan_info": (C.c_int, [P, P, P, P]),
        "mfgp_batch_mll_and_grad": (C.c_int, [P, P, P, P, OP_, P, P, P, IP, P, SZ, P]),
        "mfgp_precond_workspace_bytes": (SZ, [I32, I64, I32, I32, I32, I32, I32]),
        "mfgp_pivoted_cholesky": (C.c_int, [KP, P, I64, I32, P, P, P, SZ, P]),
        "mfgp_precond_probes": (C.c_int, [P, I64, I32, C.c_float, P, P, I32, P, P]),
        "mfgp_precond_apply": (C.c_int, [P, I64, I32, C.c_float, P, I32, P, P, P, SZ, P]),
        "mfgp_precond_cg_solve": (C.c_int, [KP, P, I64, P, I32, P, P, I32, OP_, IP, P, P, SZ, P]),
        "mfgp_precond_mll_and_grad": (C.c_int, [KP, P, I64, P, I32, P, P, I32, OP_, P, P, P, P, IP, P, SZ, P]),
        "mfgp_ski_workspace_bytes": (SZ, [I32, I64, I32, I32, C.POINTER(SkiGridT)]),
        "mfgp_ski_matvec": (C.c_int, [KP, P, I64, C.POINTER(SkiGridT), P, I32, P, P, SZ, P]),
        "mfgp_ski_cg_solve": (C.c_int, [KP, P, I64, C.POINTER(SkiGridT), P, I32, P, OP_, IP, P, SZ, P]),
        "mfgp_ski_predict_mean": (C.c_int, [KP, P, I64, P, I64, C.POINTER(SkiGridT), P, I32, P, P, SZ, P]),
        "mfgp_ski_mll_and_grad": (C.c_int, [KP, P, I64, C.POINTER(SkiGridT), P, I32, P, OP_, P, P, P, IP, P, SZ, P]),
        "mfgp_status_string": (C.c_char_p, [C.c_int]),
        "mfgp_last_hip_error": (C.c_int, []),
        "mfgp_version": (C.c_int, []),
        "mfgp_release_thread_resources": (C.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = load_library()


class MfgpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = LIB.mfgp_status_string(status).decode()
        if status == ERR_HIP:
            msg += f" (hipError {LIB.mfgp_last_hip_error()})"
        super().__init__(f"{where}: {msg}")
        self.status = status


def _check(status: int, where: str, allow=(OK,)):
    if status not in allow:
        raise MfgpError(status, where)
    return status


@dataclass
class Kernel:
    """Kernel hyperparameters: family, lengthscale (float or per-dimension), s^2, sigma^2
    and, for the periodic family, the period."""

    family: str
    lengthscale: object
    outputscale: float = 1.0
    noise: float = 0.01
    period: float = 1.0

    def struct(self, d: int) -> KernelT:
        k = KernelT()
        k.family = FAMILIES[self.family]
        k.d = d
        ls = self.lengthscale
        if isinstance(ls, (list, tuple)) or (hasattr(ls, "ndim") and getattr(ls, "ndim") == 1):
            vals = [float(v) for v in ls]
            if len(vals) != d:
                raise ValueError("ARD lengthscale needs one value per dimension")
            k.ard = 1
            for q, v in enumerate(vals):
                k.lengthscale[q] = v
        else:
            k.ard = 0
            k.lengthscale[0] = float(ls)
        k.outputscale = float(self.outputscale)
        k.noise = float(self.noise)
        k.period = float(self.period)
        return k

    def n_params(self, d: int) -> int:
        return LIB.mfgp_num_params(C.byref(self.struct(d)))

    def feature_dim(self, d: int) -> int:
        """The d of the workspace-size queries (2 d for the periodic family)."""
        return LIB.mfgp_feature_dim(C.byref(self.struct(d)))

    def __add__(self, other) -> "KernelSum":
        return KernelSum(self.terms() + other.terms())

    def __mul__(self, other) -> "KernelProd":
        return KernelProd(self.factors() + other.factors())

    def terms(self) -> list:
        return [self]

    def factors(self) -> list:
        return [self]


class KernelProd:
    """Product of kernels s2 prod_f k_f: s2 and the noise are the first
    factor's (the others' outputscale and noise are ignored).  Passed to the
    library as a chain of KernelT linked by `times`."""

    def __init__(self, factors):
        self._factors = list(factors)

    def terms(self) -> list:
        return [self]

    def factors(self) -> list:
        return list(self._factors)

    def __add__(self, other) -> "KernelSum":
        return KernelSum(self.terms() + other.terms())

    def __mul__(self, other) -> "KernelProd":
        return KernelProd(self.factors() + other.factors())

    @property
    def noise(self) -> float:
        return self._factors[0].noise

    def struct(self, d: int) -> KernelT:
        arr = (KernelT * len(self._factors))(*[k.struct(d) for k in self._factors])
        for q in range(len(self._factors) - 1):
            arr[q].times = C.pointer(arr[q + 1])
        head = arr[0]
        head._chain_ref = arr
        return head

    def n_params(self, d: int) -> int:
        return LIB.mfgp_num_params(C.byref(self.struct(d)))

    def feature_dim(self, d: int) -> int:
        return LIB.mfgp_feature_dim(C.byref(self.struct(d)))


class KernelSum:
    """Sum of kernels (each with its own parameters and outputscale); the noise
    is the first term's.  Passed to the library as a chain of KernelT."""

    def __init__(self, terms):
        self._terms = list(terms)

    def terms(self) -> list:
        return list(self._terms)

    def __add__(self, other) -> "KernelSum":
        return KernelSum(self.terms() + other.terms())

    def factors(self) -> list:
        raise TypeError("a product of a sum is not provided; expand it into a sum of products")

    @property
    def noise(self) -> float:
        return self._terms[0].noise

    def struct(self, d: int) -> KernelT:
        heads = [k.struct(d) for k in self._terms]
        arr = (KernelT * len(self._terms))(*heads)
        for q in range(len(self._terms) - 1):
            arr[q].next = C.pointer(arr[q + 1])
        head = arr[0]
        head._chain_ref = (arr, heads)   # the chains (and product factors) live as long as the head
        return head

    def n_params(self, d: int) -> int:
        return LIB.mfgp_num_params(C.byref(self.struct(d)))

    def feature_dim(self, d: int) -> int:
        return LIB.mfgp_feature_dim(C.byref(self.struct(d)))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_WS = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """Grow-only cached workspace per device (allocated by torch, not the library)."""
    key = torch.device(device)
    ws = _WS.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=key)
        _WS[key] = ws
    return ws


def workspace_bytes(op: int, n: int, d: int, t: int, precision: int = 0, max_iter: int = 0) -> int:
    return int(LIB.mfgp_workspace_bytes(op, n, d, t, precision, max_iter))


def _cols(V: torch.Tensor) -> int:
    return 1 if V.dim() == 1 else V.shape[1]


def kernel_matvec(kern: Kernel, X: torch.Tensor, V: torch.Tensor, precision: str = "fp32",
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K_y V for V [n] or [n, t] (float32)."""
    _dev(X, torch.float32, "X")
    _dev(V, torch.float32, "V")
    n, d = X.shape
    t = _cols(V)
    out = torch.empty_like(V) if out is None else _dev(out, torch.float32, "out")
    pr = PRECISIONS[precision]
    nb = workspace_bytes(OP_MATVEC, n, kern.feature_dim(d), t, pr)
    if nb == 0:
        raise MfgpError(ERR_ARG, "kernel_matvec")
    ws = workspace(nb, X.device)
    ks = kern.struct(d)
    _check(LIB.mfgp_kernel_matvec(C.byref(ks), _ptr(X), n, _ptr(V), t, _ptr(out), pr, _ptr(ws),
                                  ws.numel(), _stream()), "kernel_matvec")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20   # MFGP_NOALLOC_SCRATCH_BYTES


def kernel_matvec_noalloc(kern: Kernel, X: torch.Tensor, V: torch.Tensor, out: torch.Tensor,
                          precision: str = "fp32") -> torch.Tensor:
    """K_y V into the caller's `out` through the entry point that allocates
    nothing (the library's fixed per-GPU workspace; see the header for its
    size limit and the rule that overlapping calls on one GPU race)."""
    _dev(X, torch.float32, "X")
    _dev(V, torch.float32, "V")
    _dev(out, torch.float32, "out")
    n, d = X.shape
    t = _cols(V)
    ks = kern.struct(d)
    _check(LIB.mfgp_kernel_matvec_noalloc(C.byref(ks), _ptr(X), n, _ptr(V), t, _ptr(out),
                                          PRECISIONS[precision], _stream()), "kernel_matvec_noalloc")
    return out


def residual(kern: Kernel, X: torch.Tensor, B: torch.Tensor, Xsol: torch.Tensor):
    """(R, rel) with R = B - K_y Xsol (FP32 entries, FP64 sums); rel per column."""
    _dev(X, torch.float32, "X")
    _dev(B, torch.float32, "B")
    _dev(Xsol, torch.float64, "Xsol")
    n, d = X.shape
    t = _cols(B)
    R = torch.empty(B.shape, dtype=torch.float64, device=B.device)
    rel = (C.c_double * t)()
    ws = workspace(workspace_bytes(OP_RESIDUAL, n, kern.feature_dim(d), t), X.device)
    ks = kern.struct(d)
    _check(LIB.mfgp_residual(C.byref(ks), _ptr(X), n, _ptr(B), _ptr(Xsol), t, _ptr(R), rel,
                             _ptr(ws), ws.numel(), _stream()), "residual")
    return R, list(rel)


def cg_opts(tol: float = 1e-6, max_iter: int = 0, check_every: int = 0, max_refine: int = -1,
            precision: str = "fp32", warm_start: bool = False, probe_seed: int = 0,
            progress=None, progress_every: int = 0, replacement: bool = True, graph: bool = True) -> CgOptsT:
    """CG options; progress(iterations, rel_resid) is called during long solves."""
    o = CgOptsT()
    o.no_replacement = 0 if replacement else 1
    o.no_graph = 0 if graph else 1
    if progress is not None:
        cb = PROGRESS_FN(lambda _u, it, rr: progress(int(it), float(rr)))
        o.progress = cb
        o._cb_ref = cb   # keep the ctypes thunk alive with the options
        o.progress_every = progress_every
    o.tol = tol
    o.max_iter = max_iter
    o.check_every = check_every
    o.max_refine = max_refine
    o.precision = PRECISIONS[precision]
    o.warm_start = 1 if warm_start else 0
    o.probe_seed = probe_seed
    return o


def _info_list(info, t):
    return [dict(iters=info[c].iters, lanczos_len=info[c].lanczos_len, refinements=info[c].refinements,
                 status=info[c].status, rel_resid_recurrence=info[c].rel_resid_recurrence,
                 rel_resid_true=info[c].rel_resid_true, replacements=info[c].replacements,
                 drift_skips=info[c].drift_skips, stalls=info[c].stalls,
                 precision=PRECISION_NAMES.get(info[c].precision, info[c].precision)) for c in range(t)]


def cg_solve(kern: Kernel, X: torch.Tensor, B: torch.Tensor, tol: float = 1e-6, max_iter: int = 0,
             precision: str = "fp32", x0: Optional[torch.Tensor] = None, want_lanczos: bool = False,
             check_every: int = 0, max_refine: int = -1, allow=(OK, NOT_CONVERGED, BREAKDOWN),
             progress=None, replacement: bool = True, graph: bool = True):
    """Solve K_y X = B.  Returns (Xsol float64, info list, lanczos or None, status)."""
    _dev(X, torch.float32, "X")
    _dev(B, torch.float32, "B")
    n, d = X.shape
    t = _cols(B)
    o = cg_opts(tol, max_iter, check_every, max_refine, precision, x0 is not None, progress=progress,
                replacement=replacement, graph=graph)
    mi = max_iter if max_iter > 0 else min(max(2 * n, 64), 20000)
    Xsol = torch.zeros(B.shape, dtype=torch.float64, device=B.device) if x0 is None else \
        _dev(x0, torch.float64, "x0").clone()
    lan = torch.empty((t, mi, 2), dtype=torch.float64, device=B.device) if want_lanczos else None
    info = (CgInfoT * t)()
    ws = workspace(workspace_bytes(OP_CG, n, kern.feature_dim(d), t, o.precision, max_iter), X.device)
    ks = kern.struct(d)
    st = LIB.mfgp_cg_solve(C.byref(ks), _ptr(X), n, _ptr(B), t, _ptr(Xsol), C.byref(o), info,
                           _ptr(lan), _ptr(ws), ws.numel(), _stream())
    _check(st, "cg_solve", allow)
    return Xsol, _info_list(info, t), lan, st


def predict_mean(kern: Kernel, X: torch.Tensor, Xs: torch.Tensor, A: torch.Tensor) -> torch.Tensor:
    """mu = s2 k(Xs, X) A (no noise term)."""
    _dev(X, torch.float32, "X")
    _dev(Xs, torch.float32, "Xs")
    _dev(A, torch.float32, "A")
    n, d = X.shape
    m = Xs.shape[0]
    t = _cols(A)
    mu = torch.empty((m,) if A.dim() == 1 else (m, t), dtype=torch.float32, device=X.device)
    ws = workspace(workspace_bytes(OP_PREDICT, n, kern.feature_dim(d), t, 0, m), X.device)
    ks = kern.struct(d)
    _check(LIB.mfgp_predict_mean(C.byref(ks), _ptr(X), n, _ptr(Xs), m, _ptr(A), t, _ptr(mu), _ptr(ws),
                                 ws.numel(), _stream()), "predict_mean")
    return mu


def predict_variance(kern: Kernel, X: torch.Tensor, Xs: torch.Tensor, Z: Optional[torch.Tensor] = None,
                     num_probes: int = 64, seed: int = 0, tol: float = 1e-6, max_iter: int = 0,
                     precision: str = "fp32", allow=(OK, NOT_CONVERGED, BREAKDOWN)):
    """Latent predictive variance at Xs by the stochastic diagonal estimator on the CG path.

    Z [m, p] probes (None: seeded Rademacher, p = num_probes).  Returns
    (var float32 [m], info list, status)."""
    _dev(X, torch.float32, "X")
    _dev(Xs, torch.float32, "Xs")
    n, d = X.shape
    m = Xs.shape[0]
    if Z is not None:
        _dev(Z, torch.float32, "Z")
        p = _cols(Z)
    else:
        p = num_probes
    o = cg_opts(tol, max_iter, 0, -1, precision, False)
    o.probe_seed = seed
    var = torch.empty(m, dtype=torch.float32, device=X.device)
    info = (CgInfoT * p)()
    ws = workspace(LIB.mfgp_variance_workspace_bytes(n, kern.feature_dim(d), m, p, o.precision), X.device)
    ks = kern.struct(d)
    st = LIB.mfgp_predict_variance(C.byref(ks), _ptr(X), n, _ptr(Xs), m, p, _ptr(Z), C.byref(o), _ptr(var),
                                   info, _ptr(ws), ws.numel(), _stream())
    _check(st, "predict_variance", allow)
    return var, _info_list(info, p), st


def slq_quadrature(coeffs: Sequence[Sequence[float]], znorm2: float) -> float:
    """Host-only Gauss quadrature from CG (alpha, beta) pairs."""
    m = len(coeffs)
    buf = (C.c_double * (2 * m))(*[float(v) for ab in coeffs for v in ab])
    q = C.c_double()
    _check(LIB.mfgp_slq_quadrature(buf, m, znorm2, C.byref(q)), "slq_quadrature")
    return q.value


def mll_and_grad(kern: Kernel, X: torch.Tensor, y: torch.Tensor, num_probes: int = 16,
                 Z: Optional[torch.Tensor] = None, tol: float = 1e-6, max_iter: int = 0,
                 precision: str = "fp32", probe_seed: int = 0, want_grad: bool = True,
                 want_alpha: bool = False, allow=(OK, NOT_CONVERGED, BREAKDOWN), progress=None,
                 replacement: bool = True, check_every: int = 0, graph: bool = True):
    """Returns dict(mll, logdet, grad, alpha, info, status).

    check_every: iterations between the host's convergence checks (0: chosen
    from the product size); residual replacement runs only at 1 or 2.
    graph: replay captured iterations when the checks are 4 or more apart."""
    _dev(X, torch.float32, "X")
    _dev(y, torch.float32, "y")
    n, d = X.shape
    if Z is not None:
        _dev(Z, torch.float32, "Z")
        num_probes = Z.shape[1]
    t = num_probes + 1
    o = cg_opts(tol, max_iter, check_every, -1, precision, False, probe_seed, progress=progress,
                replacement=replacement, graph=graph)
    mi = max_iter if max_iter > 0 else min(max(2 * n, 64), 20000)
    ws = workspace(workspace_bytes(OP_MLL, n, kern.feature_dim(d), t, o.precision, mi), X.device)
    ks = kern.struct(d)
    npar = LIB.mfgp_num_params(C.byref(ks))
    mll, ld = C.c_double(), C.c_double()
    grad = (C.c_double * npar)() if want_grad else None
    alpha = torch.empty(n, dtype=torch.float64, device=X.device) if want_alpha else None
    info = (CgInfoT * t)()
    st = LIB.mfgp_mll_and_grad(C.byref(ks), _ptr(X), n, _ptr(y), num_probes, _ptr(Z), C.byref(o),
                               C.byref(mll), C.byref(ld), grad, _ptr(alpha), info, _ptr(ws),
                               ws.numel(), _stream())
    _check(st, "mll_and_grad", allow)
    return dict(mll=mll.value, logdet=ld.value, grad=None if grad is None else list(grad),
                alpha=alpha, info=_info_list(info, t), status=st)


def kernel_adjoint(kern: Kernel, X: torch.Tensor, A: torch.Tensor, B: torch.Tensor,
                   colw: Sequence[float]) -> list:
    """sum_c colw_c A_c^T (dK_y/dtheta) B_c for every parameter."""
    _dev(X, torch.float32, "X")
    _dev(A, torch.float32, "A")
    _dev(B, torch.float32, "B")
    n, d = X.shape
    t = _cols(A)
    w = (C.c_double * t)(*[float(v) for v in colw])
    ks = kern.struct(d)
    npar = LIB.mfgp_num_params(C.byref(ks))
    g = (C.c_double * npar)()
    ws = workspace(workspace_bytes(OP_ADJOINT, n, kern.feature_dim(d), t), X.device)
    _check(LIB.mfgp_kernel_adjoint(C.byref(ks), _ptr(X), n, _ptr(A), _ptr(B), t, w, g, _ptr(ws),
                                   ws.numel(), _stream()), "kernel_adjoint")
    return list(g)


def rademacher(seed: int, n: int, p: int, device="cuda") -> torch.Tensor:
    Z = torch.empty((n, p), dtype=torch.float32, device=device)
    _check(LIB.mfgp_rademacher(seed, n, p, _ptr(Z), _stream()), "rademacher")
    return Z


# ---------------------------------------------------------------- structured kernel interpolation

def ski_grid(m, lo=None, hi=None) -> SkiGridT:
    """Grid of m[k] nodes per dimension over the points' range, or over [lo, hi]."""
    g = SkiGridT()
    for k, v in enumerate(m):
        g.m[k] = int(v)
    if lo is not None:
        g.explicit_range = 1
        for k in range(len(m)):
            g.lo[k] = float(lo[k])
            g.hi[k] = float(hi[k])
    return g


def ski_matvec(kern: Kernel, X: torch.Tensor, V: torch.Tensor, grid: SkiGridT,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """(W K_UU W^T + sigma^2 I) V by structured kernel interpolation."""
    _dev(X, torch.float32, "X")
    _dev(V, torch.float32, "V")
    n, d = X.shape
    t = _cols(V)
    out = torch.empty_like(V) if out is None else _dev(out, torch.float32, "out")
    ws = workspace(LIB.mfgp_ski_workspace_bytes(OP_MATVEC, n, d, t, C.byref(grid)), X.device)
    ks = kern.struct(d)
    _check(LIB.mfgp_ski_matvec(C.byref(ks), _ptr(X), n, C.byref(grid), _ptr(V), t, _ptr(out), _ptr(ws),
                               ws.numel(), _stream()), "ski_matvec")
    return out


def ski_cg_solve(kern: Kernel, X: torch.Tensor, B: torch.Tensor, grid: SkiGridT, tol: float = 1e-6,
                 max_iter: int = 0, allow=(OK, NOT_CONVERGED, BREAKDOWN)):
    """CG on the SKI operator.  Returns (Xsol float64, info list, status)."""
    _dev(X, torch.float32, "X")
    _dev(B, torch.float32, "B")
    n, d = X.shape
    t = _cols(B)
    o = cg_opts(tol, max_iter)
    Xsol = torch.zeros(B.shape, dtype=torch.float64, device=B.device)
    info = (CgInfoT * t)()
    ws = workspace(LIB.mfgp_ski_workspace_bytes(OP_CG, n, d, t, C.byref(grid)), X.device)
    ks = kern.struct(d)
    st = LIB.mfgp_ski_cg_solve(C.byref(ks), _ptr(X), n, C.byref(grid), _ptr(B), t, _ptr(Xsol), C.byref(o), info,
                               _ptr(ws), ws.numel(), _stream())
    _check(st, "ski_cg_solve", allow)
    return Xsol, _info_list(info, t), st


def ski_predict_mean(kern: Kernel, X: torch.Tensor, Xs: torch.Tensor, A: torch.Tensor, grid: SkiGridT) -> torch.Tensor:
    """W_* K_UU W^T A (the SKI predictive mean)."""
    _dev(X, torch.float32, "X")
    _dev(Xs, torch.float32, "Xs")
    _dev(A, torch.float32, "A")
    n, d = X.shape
    m = Xs.shape[0]
    t = _cols(A)
    mu = torch.empty((m,) if A.dim() == 1 else (m, t), dtype=torch.float32, device=X.device)
    ws = workspace(LIB.mfgp_ski_workspace_bytes(OP_PREDICT, n, d, t, C.byref(grid)), X.device)
    ks = kern.struct(d)
    _check(LIB.mfgp_ski_predict_mean(C.byref(ks), _ptr(X), n, _ptr(Xs), m, C.byref(grid), _ptr(A), t, _ptr(mu),
                                     _ptr(ws), ws.numel(), _stream()), "ski_predict_mean")
    return mu


def ski_mll_and_grad(kern: Kernel, X: torch.Tensor, y: torch.Tensor, grid: SkiGridT, num_probes: int = 16,
                     Z: Optional[torch.Tensor] = None, tol: float = 1e-6, probe_seed: int = 0,
                     want_grad: bool = True, allow=(OK, NOT_CONVERGED, BREAKDOWN)):
    """SKI log marginal likelihood, log-det and gradient.  Returns dict(mll, logdet, grad, info, status)."""
    _dev(X, torch.float32, "X")
    _dev(y, torch.float32, "y")
    n, d = X.shape
    if Z is not None:
        _dev(Z, torch.float32, "Z")
        num_probes = Z.shape[1]
    t = num_probes + 1
    o = cg_opts(tol, 0, 0, -1, "fp32", False, probe_seed)
    ws = workspace(LIB.mfgp_ski_workspace_bytes(OP_MLL, n, d, t, C.byref(grid)), X.device)
    ks = kern.struct(d)
    npar = LIB.mfgp_num_params(C.byref(ks))
    mll, ld = C.c_double(), C.c_double()
    grad = (C.c_double * npar)() if want_grad else None
    info = (CgInfoT * t)()
    st = LIB.mfgp_ski_mll_and_grad(C.byref(ks), _ptr(X), n, C.byref(grid), _ptr(y), num_probes, _ptr(Z),
                                   C.byref(o), C.byref(mll), C.byref(ld), grad, info, _ptr(ws), ws.numel(),
                                   _stream())
    _check(st, "ski_mll_and_grad", allow)
    return dict(mll=mll.value, logdet=ld.value, grad=None if grad is None else list(grad),
                info=_info_list(info, t), status=st)


# ---------------------------------------------------------------- preconditioning

def precond_workspace_bytes(op: int, n: int, d: int, t: int, rank: int, precision: int = 0,
                            max_iter: int = 0) -> int:
    return int(LIB.mfgp_precond_workspace_bytes(op, n, d, t, rank, precision, max_iter))


def pivoted_cholesky(kern: Kernel, X: torch.Tensor, rank: int):
    """Rank-k pivoted Cholesky of s^2 k(X, X): (L [rank, n] float32, pivots [rank] int32)."""
    _dev(X, torch.float32, "X")
    n, d = X.shape
    L = torch.empty((rank, n), dtype=torch.float32, device=X.device)
    piv = torch.empty(rank, dtype=torch.int32, device=X.device)
    ws = workspace(precond_workspace_bytes(OP_PCHOL, n, kern.feature_dim(d), 1, rank), X.device)
    ks = kern.struct(d)
    _check(LIB.mfgp_pivoted_cholesky(C.byref(ks), _ptr(X), n, rank, _ptr(L), _ptr(piv), _ptr(ws), ws.numel(),
                                     _stream()), "pivoted_cholesky")
    return L, piv


def precond_probes(L: torch.Tensor, noise: float, E: torch.Tensor, G: torch.Tensor) -> torch.Tensor:
    """z_c = L^T-factor e_c + sqrt(noise) g_c: probes from N(0, P) (E [rank, p], G [n, p])."""
    _dev(L, torch.float32, "L")
    _dev(E, torch.float32, "E")
    _dev(G, torch.float32, "G")
    k, n = L.shape
    p = G.shape[1]
    Z = torch.empty((n, p), dtype=torch.float32, device=G.device)
    _check(LIB.mfgp_precond_probes(_ptr(L), n, k, noise, _ptr(E), _ptr(G), p, _ptr(Z), _stream()),
           "precond_probes")
    return Z


def precond_apply(L: torch.Tensor, noise: float, R: torch.Tensor):
    """(P^{-1} R, log|P|) for P = L^T-factor L + noise I."""
    _dev(L, torch.float32, "L")
    _dev(R, torch.float32, "R")
    k, n = L.shape
    t = _cols(R)
    out = torch.empty_like(R)
    ld = C.c_double()
    ws = workspace(precond_workspace_bytes(OP_PAPPLY, n, 1, t, k), R.device)
    _check(LIB.mfgp_precond_apply(_ptr(L), n, k, noise, _ptr(R), t, _ptr(out), C.byref(ld), _ptr(ws), ws.numel(),
                                  _stream()), "precond_apply")
    return out, ld.value


def precond_cg_solve(kern: Kernel, X: torch.Tensor, B: torch.Tensor, L: torch.Tensor, tol: float = 1e-6,
                     max_iter: int = 0, precision: str = "fp32", want_lanczos: bool = False,
                     check_every: int = 0, allow=(OK, NOT_CONVERGED, BREAKDOWN), progress=None):
    """Preconditioned CG on K_y X = B.  Returns (Xsol float64, info list, lanczos or None, status)."""
    _dev(X, torch.float32, "X")
    _dev(B, torch.float32, "B")
    _dev(L, torch.float32, "L")
    n, d = X.shape
    k = L.shape[0]
    t = _cols(B)
    o = cg_opts(tol, max_iter, check_every, -1, precision, False, progress=progress)
    mi = max_iter if max_iter > 0 else min(max(2 * n, 64), 20000)
    Xsol = torch.zeros(B.shape, dtype=torch.float64, device=B.device)
    lan = torch.empty((t, mi, 2), dtype=torch.float64, device=B.device) if want_lanczos else None
    info = (CgInfoT * t)()
    ws = workspace(precond_workspace_bytes(OP_PCG, n, kern.feature_dim(d), t, k, o.precision, max_iter), X.device)
    ks = kern.struct(d)
    st = LIB.mfgp_precond_cg_solve(C.byref(ks), _ptr(X), n, _ptr(B), t, _ptr(Xsol), _ptr(L), k, C.byref(o), info,
                                   _ptr(lan), _ptr(ws), ws.numel(), _stream())
    _check(st, "precond_cg_solve", allow)
    return Xsol, _info_list(info, t), lan, st


def precond_mll_and_grad(kern: Kernel, X: torch.Tensor, y: torch.Tensor, Z: torch.Tensor, L: torch.Tensor,
                         tol: float = 1e-6, max_iter: int = 0, precision: str = "fp32", want_grad: bool = True,
                         want_alpha: bool = False, allow=(OK, NOT_CONVERGED, BREAKDOWN), progress=None):
    """MLL, log-det and gradient with the pivoted-Cholesky preconditioner; Z ~ N(0, P)."""
    _dev(X, torch.float32, "X")
    _dev(y, torch.float32, "y")
    _dev(Z, torch.float32, "Z")
    _dev(L, torch.float32, "L")
    n, d = X.shape
    k = L.shape[0]
    p = Z.shape[1]
    t = p + 1
    o = cg_opts(tol, max_iter, 0, -1, precision, False, progress=progress)
    mi = max_iter if max_iter > 0 else min(max(2 * n, 64), 20000)
    ws = workspace(precond_workspace_bytes(OP_PMLL, n, kern.feature_dim(d), t, k, o.precision, mi), X.device)
    ks = kern.struct(d)
    npar = LIB.mfgp_num_params(C.byref(ks))
    mll, ld = C.c_double(), C.c_double()
    grad = (C.c_double * npar)() if want_grad else None
    alpha = torch.empty(n, dtype=torch.float64, device=X.device) if want_alpha else None
    info = (CgInfoT * t)()
    st = LIB.mfgp_precond_mll_and_grad(C.byref(ks), _ptr(X), n, _ptr(y), p, _ptr(Z), _ptr(L), k, C.byref(o),
                                       C.byref(mll), C.byref(ld), grad, _ptr(alpha), info, _ptr(ws), ws.numel(),
                                       _stream())
    _check(st, "precond_mll_and_grad", allow)
    return dict(mll=mll.value, logdet=ld.value, grad=None if grad is None else list(grad),
                alpha=alpha, info=_info_list(info, t), status=st)


def release_thread_resources() -> None:
    """Free this thread's cached rocBLAS handles and hipFFT plans."""
    _check(LIB.mfgp_release_thread_resources(), "release_thread_resources")


def timing_enable(on: bool = True) -> None:
    """Start (or stop) per-launch HIP-event timing of the entry sweeps on this thread."""
    _check(LIB.mfgp_timing_enable(1 if on else 0), "timing_enable")


SWEEP_F32, SWEEP_F64, SWEEP_ADJOINT, SWEEP_MFMA = range(4)


def timing_read(kind: int = -1) -> dict:
    """Totals since timing_enable for one sweep kind (-1: all): milliseconds, launches,
    entries and algorithmic FLOP."""
    ms, n, en, fl = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    _check(LIB.mfgp_timing_read(kind, C.byref(ms), C.byref(n), C.byref(en), C.byref(fl)), "timing_read")
    return dict(ms=ms.value, launches=n.value, entries=en.value, flops=fl.value)


def timing_phases() -> dict:
    """Host wall milliseconds of mll_and_grad's phases since timing_enable."""
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(LIB.mfgp_timing_phases(C.byref(a), C.byref(b), C.byref(c)), "timing_phases")
    return dict(cg_ms=a.value, slq_ms=b.value, adjoint_ms=c.value)


class BatchPlan:
    """A batch of independent GP problems (packed back to back) and its plan.

    kerns[b] (same family), ns[b] rows and ds[b] dims describe problem b; the
    packed inputs are X (problem b's [n_b, d_b] block after the previous
    ones), y [sum n] and Z [sum n, p] (or None for seeded probes)."""

    def __init__(self, kerns, ns, ds, num_probes: int, max_iter: int = 0, tune: bool = True,
                 use_graph: bool = True):
        self.nprob = len(ns)
        self.ns = [int(v) for v in ns]
        self.ds = [int(v) for v in ds]
        self.p = int(num_probes)
        self.t = self.p + 1
        row, xo = 0, 0
        self.row_off, self.x_off = [], []
        for n, d in zip(self.ns, self.ds):
            self.row_off.append(row)
            self.x_off.append(xo)
            row += n
            xo += n * d
        self.rows, self.xelems = row, xo
        self._n = (C.c_int64 * self.nprob)(*self.ns)
        self._ro = (C.c_int64 * self.nprob)(*self.row_off)
        self._xo = (C.c_int64 * self.nprob)(*self.x_off)
        self._k = (KernelT * self.nprob)(*[k.struct(d) for k, d in zip(kerns, self.ds)])
        self.nparams = [LIB.mfgp_num_params(C.byref(self._k[b])) for b in range(self.nprob)]
        bt = BatchT(self.nprob, 0, self._n, self._ro, self._xo, self._k)
        self._plan = C.c_void_p()
        self._destroy = LIB.mfgp_batch_plan_destroy
        _check(LIB.mfgp_batch_plan_create(C.byref(bt), self.p, max_iter, 1 if tune else 0,
                                          1 if use_graph else 0, C.byref(self._plan)), "batch_plan_create")
        self.max_iter = max_iter

    def __del__(self):
        plan = getattr(self, "_plan", None)
        destroy = getattr(self, "_destroy", None)
        if plan is not None and plan.value and destroy is not None:
            destroy(plan)
            self._plan = None

    def workspace_bytes(self) -> int:
        return int(LIB.mfgp_batch_workspace_bytes(self._plan))

    def info(self) -> dict:
        tj, gl, ms = C.c_int64(), C.c_int64(), C.c_double()
        _check(LIB.mfgp_batch_plan_info(self._plan, C.byref(tj), C.byref(ms), C.byref(gl)), "batch_plan_info")
        return dict(tile_j=tj.value, tuned_sweep_ms=ms.value, graph_launches=gl.value)

    def mll_and_grad(self, X: torch.Tensor, y: torch.Tensor, Z: Optional[torch.Tensor] = None,
                     tol: float = 1e-6, probe_seed: int = 0, want_grad: bool = True,
                     allow=(OK, NOT_CONVERGED, BREAKDOWN), progress=None,
                     replacement: bool = True, check_every: int = 0, precision: str = "fp32") -> dict:
        _dev(X, torch.float32, "X")
        _dev(y, torch.float32, "y")
        if Z is not None:
            _dev(Z, torch.float32, "Z")
        o = cg_opts(tol, self.max_iter, check_every, -1, precision, False, probe_seed, progress=progress,
                    replacement=replacement)
        mll = (C.c_double * self.nprob)()
        ld = (C.c_double * self.nprob)()
        grad = (C.c_double * sum(self.nparams))() if want_grad else None
        info = (CgInfoT * (self.nprob * self.t))()
        ws = workspace(self.workspace_bytes(), X.device)
        st = LIB.mfgp_batch_mll_and_grad(self._plan, _ptr(X), _ptr(y), _ptr(Z), C.byref(o), mll, ld, grad,
                                         info, _ptr(ws), ws.numel(), _stream())
        _check(st, "batch_mll_and_grad", allow)
        grads, off = [], 0
        if grad is not None:
            for npar in self.nparams:
                grads.append(list(grad[off:off + npar]))
                off += npar
        infos = _info_list(info, self.nprob * self.t)
        return dict(mll=list(mll), logdet=list(ld), grad=grads if want_grad else None,
                    info=[infos[b * self.t:(b + 1) * self.t] for b in range(self.nprob)], status=st)


# ---------------------------------------------------------------- autograd

def _kernel_from_params(family: str, params: torch.Tensor, d: int, ard: bool) -> Kernel:
    th = [float(v) for v in params.detach().cpu().tolist()]
    nl = d if ard else 1
    ls = th[:nl] if ard else th[0]
    if family == "periodic":
        return Kernel(family, ls, th[nl + 1], th[nl + 2], period=th[nl])
    return Kernel(family, ls, th[nl], th[nl + 1])


class KernelMatvec(torch.autograd.Function):
    """KV = K_y(theta) V with gradients for V and theta.

    params: CPU float64 tensor [l_1..l_d (or l), (period,) s2, sigma^2].  backward:
    grad_V = K_y G (K_y is symmetric) and grad_theta[p] = sum_c G_c^T
    (dK_y/dtheta_p) V_c, both computed by the library (matrix-free product and
    adjoint sweep)."""

    @staticmethod
    def forward(ctx, V: torch.Tensor, X: torch.Tensor, params: torch.Tensor, family: str, ard: bool):
        kern = _kernel_from_params(family, params, X.shape[1], ard)
        ctx.save_for_backward(V, X)
        ctx.kern = kern
        ctx.params_meta = (params.dtype, params.device, params.shape)
        return kernel_matvec(kern, X, V.contiguous())

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        V, X = ctx.saved_tensors
        G = G.contiguous()
        gV = kernel_matvec(ctx.kern, X, G) if ctx.needs_input_grad[0] else None
        gp = None
        if ctx.needs_input_grad[2]:
            t = 1 if V.dim() == 1 else V.shape[1]
            g = kernel_adjoint(ctx.kern, X, G.reshape(V.shape[0], t).contiguous(),
                               V.reshape(V.shape[0], t).contiguous(), [1.0] * t)
            dt, dv, shp = ctx.params_meta
            gp = torch.tensor(g, dtype=dt, device=dv).reshape(shp)
        return gV, None, gp, None, None


class MarginalLogLikelihood(torch.autograd.Function):
    """log p(y | X, theta) by CG + stochastic Lanczos, differentiable in theta.

    params: CPU float64 tensor [l.. , (period,) s2, sigma^2]; Z: probes [n, p] (GPU).
    forward returns a float64 scalar; backward returns grad_out times the
    library's adjoint-sweep gradient (same probes)."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, X: torch.Tensor, y: torch.Tensor, Z: torch.Tensor,
                family: str, ard: bool, tol: float = 1e-6):
        kern = _kernel_from_params(family, params, X.shape[1], ard)
        r = mll_and_grad(kern, X, y, Z=Z, tol=tol)
        ctx.grad = torch.tensor(r["grad"], dtype=params.dtype, device=params.device).reshape(params.shape)
        return torch.tensor(r["mll"], dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return g.to(ctx.grad.dtype) * ctx.grad, None, None, None, None, None, None


LOG_2PI = math.log(2.0 * math.pi)
