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

from oracle import rng as R
from oracle import sketch as S
from oracle import slse as OS
from slse_inputs import fingerprint, make_problem, sketch_seed

from bounds import bf16_uncertain

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


U32 = 2.0 ** -24
_PROBLEMS = {}


def problem(name):
    """The regenerated workload, kept for the other tests of this module."""
    if name not in _PROBLEMS:
        _PROBLEMS[name] = make_problem(name)
    return _PROBLEMS[name]


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
    p = problem(name)
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


def test_full_workload_sketches(G):
    """Sampled outputs of the three sketches on the full mixed workload (2^22 x
    512, FP32), made by the calls and shapes bench.py times, against the oracle
    computed output by output on a sample of columns (each column of a sketch
    depends only on that column of [X|Y]).  Every bound is the worst case of
    the device's FP32 summation order over the summed terms' magnitudes."""
    p = problem("mixed")
    N, d = p.X.shape
    seed = sketch_seed("mixed")
    m = G.paper_schedule(N, d)
    r = 6 * d
    g = np.random.default_rng(7)
    cols = sorted({0, 1, d // 2, d - 1, *g.integers(0, d, 3).tolist()})
    ocols = cols + [d]  # the sampled columns of X, then Y
    Xs = p.X[:, cols]
    W = np.concatenate([Xs.astype(np.float64), p.Y.astype(np.float64)[:, None]], axis=1)
    aW = np.abs(W)
    X, Y = dev(p.X), dev(p.Y)

    # SRHT (levels as prefixes of the m_K sampled rows, bench: [m_K], r): each
    # output is a +-1 sum of every row, formed by 22 butterfly stages in FP32
    print("[sketches] srht", flush=True)
    A, Ah, lay = G.sketch_apply(X, Y, "srht", seed, [m[-1]], r)
    pw, n_pad = S.pad_pow2(N)
    sigma, sigma_hat = S.srht_orders(seed, pw, m[-1], r)
    ta = np.array([0, 1, m[-1] - 1, *g.integers(0, m[-1], 3)])
    th = np.array([0, r - 1, *g.integers(0, r, 2)])
    ref = S.srht_rows(Xs, p.Y, seed, np.concatenate([sigma[ta], sigma_hat[th]]))
    got = np.concatenate([A[torch.from_numpy(ta)][:, ocols].cpu().numpy(),
                          Ah[torch.from_numpy(th)][:, ocols].cpu().numpy()])
    tol = pw * U32 * aW.sum(axis=0)[None, :]
    assert np.all(np.abs(got - ref) <= tol), np.max(np.abs(got - ref) / tol)
    assert np.all(np.abs(ref).max(axis=0) > 10 * tol[0])  # the check is not vacuous
    del A, Ah

    # CountSketch (every level and every Hessian bucket of the sampled columns)
    print("[sketches] countsketch", flush=True)
    A, Ah, lay = G.sketch_apply(X, Y, "countsketch", seed, m, r)
    h, sg = R.countsketch_hash(seed, N, m[-1])
    hh, sh = R.countsketch_hash_hat(seed, N, r)
    sW = sg[:, None].astype(np.float64) * W
    outs = [(A[o:o + v][:, ocols].cpu().numpy(), h & (v - 1), v, sW) for o, v in zip(lay["offset"], m)]
    outs.append((Ah[:, ocols].cpu().numpy(), hh, r, sh[:, None].astype(np.float64) * W))
    for got, b, nb, terms in outs:
        cnt = np.bincount(b, minlength=nb).astype(np.float64)
        ref = np.stack([np.bincount(b, weights=terms[:, c], minlength=nb) for c in range(len(ocols))], 1)
        mag = np.stack([np.bincount(b, weights=aW[:, c], minlength=nb) for c in range(len(ocols))], 1)
        tol = (cnt[:, None] + 1) * U32 * mag
        assert np.all(np.abs(got - ref) <= tol), (nb, np.max(np.abs(got - ref) - tol))
        if nb == m[0]:  # about 1000 rows a bucket: the bound is far below the sums
            assert np.median(np.abs(ref)) > 100 * np.median(tol)
    del A, Ah

    # Gaussian, BF16 operands on the matrix cores, in bench's call (m = r =
    # 3072, the full-size launch and its data-row splits), on [X|Y] kept at a
    # few hundred rows of the workload (the first and last rows, both sides of
    # every split boundary, random rows) and zero elsewhere.  Products and
    # sums of zeros are exact, so only the kept rows' terms round: with
    # T = sum_j |G_kj| |W_jc| over them, |error| <= n_add u T (n_add as in the
    # split tests, over the kept rows) plus one BF16 ulp for each entry of G
    # whose FP64 value lies within 2^-16 (1 + |G|) of a rounding midpoint (the
    # device draws G in FP32).  Tight enough that any one row missing or
    # misplaced fails: every entry is checked.
    print("[sketches] gaussian", flush=True)
    splits = G.debug_gaussian_plan(N, d, r, True)
    per = -(-(-(-N // splits)) // 64) * 64
    edges = [s * per for s in range(1, splits) if s * per < N]
    keep = np.array(sorted({0, N - 1, *(e - 1 for e in edges), *edges,
                            *g.integers(0, N, 128).tolist()}), dtype=np.int64)
    kt = torch.from_numpy(keep).to("cuda:0")
    Xz = torch.zeros_like(X)
    Yz = torch.zeros_like(Y)
    Xz[kt] = X[kt]
    Yz[kt] = Y[kt]
    del X, Y
    A, Ah, lay = G.sketch_apply(Xz, Yz, "gaussian", seed, [r], r, bf16=True)
    Wk = S.round_to(S.joint(p.X[keep], p.Y[keep]), "bf16")
    n_add = len(keep) * 17 // 16 + splits + 16
    for out, stream in ((A, R.STREAM_G), (Ah, R.STREAM_GHAT)):
        g64 = R.gaussian_block(seed, stream, np.arange(r), keep)
        gq = S.round_to(g64, "bf16")
        unc, ulp = bf16_uncertain(g64, 2.0 ** -16 * (1.0 + np.abs(g64)))
        ref = gq @ Wk
        tol = n_add * U32 * (np.abs(gq) @ np.abs(Wk)) + np.where(unc, ulp, 0.0) @ np.abs(Wk) + 1e-300
        err = np.abs(out.cpu().numpy() - ref)
        assert np.all(err <= tol), (stream, float((err / tol).max()))
        # one row's terms (the first row of the last split) exceed the bound
        i_last = int(np.searchsorted(keep, edges[-1]))
        one = np.abs(gq[:, i_last:i_last + 1] @ Wk[i_last:i_last + 1])
        assert np.mean(one > tol) > 0.5
