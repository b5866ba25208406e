"""torch.autograd.Function wrappers: gradients through the library's adjoint.

KernelMatvec: the backward (grad_V = K_y G, grad_theta from the adjoint sweep)
is compared with central finite differences of the oracle's FP64 product and
with the oracle's bilinear form.  MarginalLogLikelihood: backward equals the
same-probe oracle gradient and the library's own gradient.
"""

import numpy as np
import pytest
import torch

from oracle import gp, krylov
from paper_2605_17898_amd import inputs
from tests.gpu_util import banner, dev, okern

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_2605_17898_amd import mfgp
    return mfgp


@pytest.mark.parametrize("family,ard", [("rbf", True), ("matern52", False), ("matern32", True)])
def test_kernel_matvec_backward(mf, family, ard):
    banner(f"KernelMatvec backward family={family} ard={ard} n=900 t=3")
    w = inputs.random_problem(91, 900, 3, family, ard=ard, noise=0.04)
    k = okern(w)
    th = torch.tensor(k.params(3), dtype=torch.float64, requires_grad=True)
    V = torch.from_numpy(inputs.gaussian_rhs(1, w.n, 3)).cuda().requires_grad_(True)
    G = inputs.gaussian_rhs(2, w.n, 3)
    out = mf.KernelMatvec.apply(V, dev(w.X), th, family, ard)
    out.backward(dev(G))
    # grad_V = K_y G
    ref_gV = gp.ky_matvec(k, w.X, G)
    assert np.linalg.norm(V.grad.cpu().numpy() - ref_gV) / np.linalg.norm(ref_gV) <= 1e-5
    # grad_theta = sum_c G_c^T dK_y V_c  (oracle bilinear form and central FD of the oracle)
    Vn = V.detach().cpu().numpy()
    ref = gp.adjoint_bilinear(k, w.X, G, Vn, [1.0, 1.0, 1.0])
    g = th.grad.numpy()
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-4
    p0 = k.params(3)
    fd = []
    for q in range(len(p0)):
        h = 1e-6 * p0[q]
        tp, tm = p0.copy(), p0.copy()
        tp[q] += h
        tm[q] -= h
        f = lambda pp: float(np.sum(G * gp.ky_matvec(k.with_params(pp), w.X, Vn)))
        fd.append((f(tp) - f(tm)) / (2 * h))
    assert np.linalg.norm(g - np.array(fd)) / np.linalg.norm(fd) <= 1e-4


def test_mll_function_backward(mf):
    banner("MarginalLogLikelihood backward, exact1k n=800 p=16")
    w = inputs.exact1k(n=800, probes=16)
    k = okern(w)
    th = torch.tensor(k.params(2), dtype=torch.float64, requires_grad=True)
    mll = mf.MarginalLogLikelihood.apply(th, dev(w.X), dev(w.y), dev(w.Z), "rbf", False)
    (2.0 * mll).backward()
    g_ref = gp.same_probe_grad(k, w.X, w.y, w.Z)
    g = th.grad.numpy() / 2.0
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) <= 1e-3
    A = gp.ky_matrix(k, w.X)
    ld = float(krylov.quadform_log(A, w.Z).mean())
    alpha = gp.solve(k, w.X, w.y)
    ref = -0.5 * (float(w.y.astype(np.float64) @ alpha) + ld + w.n * np.log(2 * np.pi))
    assert float(mll) == pytest.approx(ref, rel=1e-4)
