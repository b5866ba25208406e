"""Helpers shared by the GPU parity tests (marshalling only)."""

import numpy as np
import torch

from oracle import gp


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def okern(w, family=None, lengthscale=None):
    return gp.Kern(family or w.family, w.lengthscale if lengthscale is None else lengthscale,
                   w.outputscale, w.noise)


def mkern(w, family=None, lengthscale=None):
    from paper_2605_17898_amd import mfgp
    ls = w.lengthscale if lengthscale is None else lengthscale
    if isinstance(ls, np.ndarray):
        ls = [float(v) for v in ls]
    return mfgp.Kernel(family or w.family, ls, w.outputscale, w.noise)


def col_rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    return np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)
