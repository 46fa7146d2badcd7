"""Full-size workloads on the GPU, in the configuration bench.py times.

The solve is checked against the stored FP64 oracle solution of the same
regenerated data, and sampled columns of the fused residual gradient (the
stage-2 sweep kernel with its autotuned launch) against an FP64 host
computation over every row, within a bound derived from the magnitudes of the
summed terms.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import slse as OS
from slse_inputs import fingerprint, make_problem, sketch_seed

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


def host_grad_columns(X, Y, beta, cols, block=1 << 18):
    """FP64 g_j = sum_i X_ij (Y_i - x_i . beta) for the columns `cols`, the
    residual norm^2, and the magnitudes sum_i |X_ij| (|Y_i| + |x_i| . |beta|)
    and sum_i (|Y_i| + |x_i| . |beta|)^2 that bound their rounding errors."""
    g = np.zeros(len(cols))
    mag = np.zeros(len(cols))
    rn = 0.0
    rn_mag = 0.0
    ab = np.abs(beta)
    for i0 in range(0, X.shape[0], block):
        Xb = X[i0:i0 + block].astype(np.float64)
        Yb = Y[i0:i0 + block].astype(np.float64)
        r = Yb - Xb @ beta
        s = np.abs(Yb) + np.abs(Xb) @ ab
        Xc = Xb[:, cols]
        g += Xc.T @ r
        mag += np.abs(Xc).T @ s
        rn += r @ r
        rn_mag += s @ s
    return g, mag, rn, rn_mag


@pytest.mark.parametrize("name", ["mixed", "illcond"])
def test_full_workload_solve_and_gradient(G, name):
    with open(os.path.join(GOLDEN, f"ref_{name}.json")) as f:
        ref = json.load(f)
    p = make_problem(name)
    assert fingerprint(p.X, p.Y) == ref["fingerprint"]
    print(f"[{name}] N={p.n} d={p.d} {p.X.dtype}", flush=True)
    bstar = np.asarray(ref["beta_star"])
    X, Y = dev(p.X), dev(p.Y)
    m = G.paper_schedule(p.n, p.d)
    precision = "mixed" if p.X.dtype == np.float32 else "f64"
    prm = G.Params(kind="srht", seed=sketch_seed(name), m=m, a=[2] * len(m), r=6 * p.d,
                   s_max=40, precision=precision)
    beta, info = G.solve(X, Y, prm)
    assert info["status"] == "SLSE_OK"
    assert OS.rel_err(beta.cpu().numpy(), bstar) < 1e-10

    # the sweep kernel away from the solution (a residual with structure)
    b = bstar + 1e-3 * np.random.default_rng(5).standard_normal(p.d)
    g, rn = G.fused_resid_grad(X, Y, dev(b))
    cols = sorted({0, 1, p.d // 2, p.d - 1, *np.random.default_rng(6).integers(0, p.d, 4).tolist()})
    gref, mag, rnref, rn_mag = host_grad_columns(p.X, p.Y, b, cols)
    # both sides accumulate in FP64: each residual is a dot of d + 1 terms and
    # each column a sum of N products, so the rounding stays below
    # (d + 1 + log2-depth and per-lane chain lengths) u |terms|; 2e-12 covers
    # both sides with room, far below |g_j| (a dropped or misplaced term
    # moves g_j by O(|x| |r|) per row)
    err = np.abs(g.cpu().numpy()[cols] - gref)
    assert np.all(err <= 2e-12 * mag), (cols, err, mag)
    assert np.all(np.abs(gref) > 1e3 * 2e-12 * mag)  # the check is not vacuous
    assert abs(rn.item() - rnref) <= 2e-12 * rn_mag
