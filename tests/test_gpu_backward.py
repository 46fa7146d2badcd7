"""GPU adjoint (slse_backward / SLSEFunction) against the oracle.

Full size: the backward workload (N = 2^20, d = 256, FP32 data) against the
stored oracle lambda and beta_star (tests/golden/ref_backward.json), the
reference gradients formed from them in FP64.  Small: a 4096 x 16 slice
against the oracle adjoint and against central finite differences of
w^T beta_hat on sampled entries.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import adjoint as ADJ
from oracle import slse as OS
from slse_inputs import fingerprint, make_problem
from slse_inputs.generators import loss_vector

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_06856_amd import slse

    return slse


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _params(G, n, d, s_max=40, precision="mixed"):
    m = G.paper_schedule(n, d)
    return G.Params(kind="srht", seed=1004, m=m, a=[2] * len(m), r=6 * d, s_max=s_max,
                    precision=precision)


def test_backward_full_workload_against_reference(G):
    with open(os.path.join(GOLDEN, "ref_backward.json")) as f:
        ref = json.load(f)
    p = make_problem("backward")
    assert fingerprint(p.X, p.Y) == ref["fingerprint"]
    bstar = np.asarray(ref["beta_star"])
    lam = np.asarray(ref["lambda"])
    w = np.asarray(ref["w"])
    assert np.array_equal(w, loss_vector(p.d))
    X, Y = dev(p.X), dev(p.Y)
    prm = _params(G, p.n, p.d)
    beta, _ = G.solve(X, Y, prm)
    assert OS.rel_err(beta.cpu().numpy(), bstar) < 1e-10
    dX, dY, glam = G.backward(X, Y, prm, beta, dev(w), grad_dtype=torch.float64)
    assert OS.rel_err(glam.cpu().numpy(), lam) < 1e-9
    Xd = p.X.astype(np.float64)
    u = Xd @ lam
    r = p.Y.astype(np.float64) - Xd @ bstar
    rY = u
    e_dY = np.linalg.norm(dY.cpu().numpy() - rY) / np.linalg.norm(rY)
    dXg = dX.cpu().numpy()
    num = np.sqrt(np.sum((dXg - (np.outer(r, lam) - np.outer(u, bstar))) ** 2))
    den = np.sqrt(np.sum((np.outer(r, lam) - np.outer(u, bstar)) ** 2))
    assert e_dY < 1e-6 and num / den < 1e-6
    # FP32 gradients: within FP32 rounding of the FP64 ones
    dX32, dY32, _ = G.backward(X, Y, prm, beta, dev(w))
    assert dX32.dtype == torch.float32
    assert np.linalg.norm(dX32.cpu().numpy() - dXg) / np.linalg.norm(dXg) < 1e-6


def test_backward_slice_matches_oracle_and_finite_differences(G):
    p = make_problem("backward", n=4096, d=16)
    X64 = p.X.astype(np.float64)
    Y64 = p.Y.astype(np.float64)
    w = np.random.default_rng(8).standard_normal(16)
    prm = _params(G, 4096, 16, s_max=40, precision="f64")
    X, Y = dev(X64), dev(Y64)
    beta, _ = G.solve(X, Y, prm)
    dX, dY, _ = G.backward(X, Y, prm, beta, dev(w))
    rX, rY, _, _ = ADJ.adjoint(X64, Y64, w)
    assert np.linalg.norm(dX.cpu().numpy() - rX) / np.linalg.norm(rX) < 1e-9
    assert np.linalg.norm(dY.cpu().numpy() - rY) / np.linalg.norm(rY) < 1e-9
    # central differences on sampled entries (FP64, h ~ 6e-6 scale)
    rng = np.random.default_rng(1)
    gX = dX.cpu().numpy()
    gY = dY.cpu().numpy()
    for _ in range(12):
        i, j = int(rng.integers(4096)), int(rng.integers(16))
        h = 6e-6 * max(1.0, abs(X64[i, j]))
        Xp, Xm = X64.copy(), X64.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        fd = (w @ ADJ._ols_solve(Xp, Y64) - w @ ADJ._ols_solve(Xm, Y64)) / (2 * h)
        assert abs(fd - gX[i, j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7
        h = 6e-6 * max(1.0, abs(Y64[i]))
        Yp, Ym = Y64.copy(), Y64.copy()
        Yp[i] += h
        Ym[i] -= h
        fd = (w @ ADJ._ols_solve(X64, Yp) - w @ ADJ._ols_solve(X64, Ym)) / (2 * h)
        assert abs(fd - gY[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7


def test_autograd_function(G):
    p = make_problem("backward", n=8192, d=12)
    X = dev(p.X.astype(np.float64)).requires_grad_(True)
    Y = dev(p.Y.astype(np.float64)).requires_grad_(True)
    w = torch.from_numpy(np.random.default_rng(3).standard_normal(12)).to("cuda:0")
    prm = _params(G, 8192, 12, s_max=40, precision="f64")
    beta = G.SLSEFunction.apply(X, Y, prm)
    loss = (beta * w).sum()
    loss.backward()
    rX, rY, _, _ = ADJ.adjoint(p.X.astype(np.float64), p.Y.astype(np.float64), w.cpu().numpy())
    assert np.linalg.norm(X.grad.cpu().numpy() - rX) / np.linalg.norm(rX) < 1e-9
    assert np.linalg.norm(Y.grad.cpu().numpy() - rY) / np.linalg.norm(rY) < 1e-9
