"""GPU parity of libslse's kernels against the CPU oracle (through the C ABI).

Integer streams (Philox words, permutations, signs, hashes) must match bit for
bit.  Floating-point results are compared element by element against the
oracle on the same seeded inputs, with bounds derived from the arithmetic:
  * fused residual gradient: |g - g_ref| <= c u_acc B with
    B_k = sum_j |x_jk| (|y_j| + |x_j| . |beta|), c = d + n/4096 + 64
    (d-term dot, sequential per-lane sums, then a reduction tree);
  * Walsh-Hadamard sketch: |A - A_ref| <= 2 (p + 1) u_T sum_j |w_jc| per column
    (p butterfly additions per output, every one bounded by the column's l1 norm).
"""
import os

import numpy as np
import pytest
import torch

from oracle import adjoint as ADJ
from oracle import ols as O
from oracle import rng as R
from oracle import sketch as S
from oracle import slse as OS
from slse_inputs import make_problem

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_06856_amd import slse

    return slse


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# ---------------------------------------------------------------------------
# counter streams: bit-exact
# ---------------------------------------------------------------------------
def test_philox_words_bit_exact(G):
    start = 2 ** 40 + 12345
    out = G.debug_stream(0, 123456789, 5, 77, start, 5000).cpu().numpy().view(np.uint64)
    out = out.reshape(-1, 4)
    c = np.arange(start, start + 5000, dtype=np.uint64)
    ref = R.philox4x64(c, 77, 0, 0, 123456789, 5)
    for k in range(4):
        assert np.array_equal(out[:, k], ref[k])


@pytest.mark.parametrize("p", [1, 2, 5, 10, 13, 20, 21])
def test_permutations_bit_exact(G, p):
    n = min(1 << p, 1 << 15)
    start = (1 << p) - n
    x = np.arange(start, start + n)
    for stream in (R.STREAM_P, R.STREAM_S, R.STREAM_SHAT):
        fwd = G.debug_stream(1, 99, stream, p, start, n).cpu().numpy()
        inv = G.debug_stream(2, 99, stream, p, start, n).cpu().numpy()
        assert np.array_equal(fwd, R.prp(x, 99, stream, p).astype(np.int64))
        assert np.array_equal(inv, R.prp_inverse(x, 99, stream, p).astype(np.int64))


def test_signs_and_hashes_bit_exact(G):
    n = 100000
    D = G.debug_stream(3, 7, 0, 0, 0, n).cpu().numpy()
    assert np.array_equal(D, R.rademacher(7, n).astype(np.int64))
    h = G.debug_stream(4, 7, 0, 1024, 0, n).cpu().numpy()
    s = G.debug_stream(5, 7, 0, 1024, 0, n).cpu().numpy()
    hr, sr = R.countsketch_hash(7, n, 1024)
    assert np.array_equal(h, hr) and np.array_equal(s, sr.astype(np.int64))
    hh = G.debug_stream(6, 7, 0, 192, 0, n).cpu().numpy()
    sh = G.debug_stream(7, 7, 0, 192, 0, n).cpu().numpy()
    hhr, shr = R.countsketch_hash_hat(7, n, 192)
    assert np.array_equal(hh, hhr) and np.array_equal(sh, shr.astype(np.int64))


def test_gaussian_entries_match_box_muller(G):
    g = G.debug_gaussian(11, 7, 0, 64, 1000, 500).cpu().numpy()
    ref = R.gaussian_block(11, 7, np.arange(64), np.arange(1000, 1500))
    diff = np.abs(g - ref)
    # FP32 Box-Muller: ~1e-6 relative; near u1 -> 1 the radius is tiny and its
    # absolute error is bounded by ~1e-3
    assert np.quantile(diff / np.maximum(1.0, np.abs(ref)), 0.999) < 2e-6
    assert diff.max() < 1e-3


# ---------------------------------------------------------------------------
# fused residual gradient
# ---------------------------------------------------------------------------
def _grad_bound(Xd, Yd, beta, u, scale):
    n, d = Xd.shape
    B = np.abs(Xd).T @ (np.abs(Yd) + np.abs(Xd) @ np.abs(beta))
    c = d + n / 4096 + 64
    return c * u * abs(scale) * B + 1e-300


@pytest.mark.parametrize("dtype,accum", [(np.float64, "f64"), (np.float32, "f64"),
                                         (np.float32, "f32"), (np.float64, "f32")])
@pytest.mark.parametrize("n,d", [(1, 3), (1000, 33), (70001, 256), (20000, 512), (5000, 17),
                                 (3000, 1), (40000, 64)])
def test_fused_resid_grad_parity(G, n, d, dtype, accum):
    g = np.random.default_rng(n + d)
    X = g.standard_normal((n, d)).astype(dtype)
    Y = g.standard_normal(n).astype(dtype)
    beta = g.standard_normal(d)
    gg, rn = G.fused_resid_grad(dev(X), dev(Y), dev(beta), scale=0.5, accum=accum)
    Xd = X.astype(np.float64)
    Yd = Y.astype(np.float64)
    ref = 0.5 * OS.full_grad(Xd, Yd, beta)
    u = U64 if accum == "f64" else U32
    bound = _grad_bound(Xd, Yd, beta, u, 0.5)
    assert np.all(np.abs(gg.cpu().numpy() - ref) <= bound)
    r = Yd - Xd @ beta
    assert abs(rn.item() - 0.5 * r @ r) <= (d + n / 4096 + 64) * u * 0.5 * ((np.abs(Yd) + np.abs(Xd) @ np.abs(beta)) ** 2).sum()


@pytest.mark.parametrize("dtype,d,lpr", [(np.float32, 512, 16), (np.float32, 512, 64),
                                         (np.float32, 128, 32), (np.float64, 256, 8),
                                         (np.float64, 64, 32)])
@pytest.mark.parametrize("blocks", [7, 256])
def test_fused_resid_grad_whole_vector_path(G, dtype, d, lpr, blocks, monkeypatch):
    # rows that split into whole vectors take the unguarded main loop; the row
    # count leaves a ragged tail in every block, and the result matches both
    # the oracle and the guarded path
    monkeypatch.setenv("SLSE_RG_LPR", str(lpr))
    monkeypatch.setenv("SLSE_RG_BLOCKS", str(blocks))
    n = 30011
    g = np.random.default_rng(d + lpr)
    X = g.standard_normal((n, d)).astype(dtype)
    Y = g.standard_normal(n).astype(dtype)
    beta = g.standard_normal(d)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    ref = OS.full_grad(Xd, Yd, beta)
    bound = _grad_bound(Xd, Yd, beta, U64, 1.0)
    g_full, _ = G.fused_resid_grad(dev(X), dev(Y), dev(beta))
    monkeypatch.setenv("SLSE_RG_FULL", "0")
    g_guard, _ = G.fused_resid_grad(dev(X), dev(Y), dev(beta))
    assert np.all(np.abs(g_full.cpu().numpy() - ref) <= bound)
    assert np.all(np.abs(g_guard.cpu().numpy() - ref) <= bound)


def test_fused_resid_grad_padded_ld_null_y_and_empty(G):
    g = np.random.default_rng(5)
    Xw = g.standard_normal((9000, 40))
    X = dev(Xw)[:, :37]  # ldx = 40 > d
    beta = g.standard_normal(37)
    gg, _ = G.fused_resid_grad(X, None, dev(beta))
    ref = OS.full_grad(Xw[:, :37], np.zeros(9000), beta)
    assert np.all(np.abs(gg.cpu().numpy() - ref) <= _grad_bound(Xw[:, :37], np.zeros(9000), beta, U64, 1.0))
    g0, r0 = G.fused_resid_grad(X, None, dev(beta), n=0)
    assert np.all(g0.cpu().numpy() == 0) and r0.item() == 0


def test_fused_resid_grad_is_deterministic(G):
    g = np.random.default_rng(9)
    X = dev(g.standard_normal((123457, 96)))
    Y = dev(g.standard_normal(123457))
    b = dev(g.standard_normal(96))
    a1, _ = G.fused_resid_grad(X, Y, b)
    a2, _ = G.fused_resid_grad(X, Y, b)
    assert torch.equal(a1, a2)


# ---------------------------------------------------------------------------
# sketches
# ---------------------------------------------------------------------------
def _srht_bound(X, Y, p, u):
    W = S.joint(X, Y)
    return 2 * (p + 1) * u * np.abs(W).sum(axis=0)[None, :] + 1e-300


@pytest.mark.parametrize("N,d,dtype,m,r,bmax", [
    (1000, 5, np.float64, [16, 32, 64], 24, None),        # N' = 1024, one pass
    (16384, 32, np.float64, [64, 128, 256, 512, 1024], 192, None),  # two passes
    (5000, 7, np.float32, [64, 128], 48, None),
    (70000, 63, np.float64, [1024, 2048, 4096], 400, None),
    (70000, 63, np.float64, [1024, 2048, 4096], 400, 11),  # two passes of 9 and 8 stages
    (3, 1, np.float64, [2, 4], 3, None),                   # tiny: N' = 4
    (2000, 40, np.float32, [256, 512], 90, None),          # one 11-stage pass, two LDS rounds
    (2000, 20, np.float64, [256, 512], 60, 11),            # the same for FP64
    (5000, 33, np.float32, [512, 1024], 80, 7),            # three passes of 5, 4, 4 stages
])
def test_srht_parity(G, N, d, dtype, m, r, bmax, monkeypatch):
    if bmax:
        monkeypatch.setenv("SLSE_SRHT_BMAX", str(bmax))
    g = np.random.default_rng(N + d)
    X = g.standard_normal((N, d)).astype(dtype)
    Y = g.standard_normal(N).astype(dtype)
    A, Ah, lay = G.sketch_apply(dev(X), dev(Y), "srht", 4242, m, r)
    ref = S.srht(X.astype(np.float64), Y.astype(np.float64), 4242, m, r)
    p = int(np.log2(ref["n_pad"]))
    u = U64 if dtype == np.float64 else U32
    bound = _srht_bound(X.astype(np.float64), Y.astype(np.float64), p, u)
    assert np.all(np.abs(A.cpu().numpy() - ref["A"]) <= bound)
    assert np.all(np.abs(Ah.cpu().numpy() - ref["Ahat"]) <= bound)
    assert lay["scale"] == ref["scale"] and lay["hat_scale"] == ref["hat_scale"]
    assert lay["n_pad"] == ref["n_pad"]


@pytest.mark.slow
def test_srht_three_passes(G):
    N, d = (1 << 21) - 5, 3
    g = np.random.default_rng(1)
    X = g.standard_normal((N, d))
    Y = g.standard_normal(N)
    A, Ah, lay = G.sketch_apply(dev(X), dev(Y), "srht", 77, [4096, 8192], 64)
    rows = [0, 1, 777, 8191]
    sigma, sigma_hat = S.srht_orders(77, 21, 8192, 64)
    ref = S.srht_rows(X, Y, 77, np.concatenate([sigma[rows], sigma_hat[[0, 63]]]))
    bound = _srht_bound(X, Y, 21, U64)
    assert np.all(np.abs(A.cpu().numpy()[rows] - ref[:4]) <= bound)
    assert np.all(np.abs(Ah.cpu().numpy()[[0, 63]] - ref[4:]) <= bound)


@pytest.mark.slow
def test_srht_two_eleven_stage_passes(G):
    # FP32 with N' = 2^22: two passes of 11 stages, each exchanging its tile in two LDS rounds
    N, d = (1 << 22) - 9, 2
    g = np.random.default_rng(5)
    X = g.standard_normal((N, d)).astype(np.float32)
    Y = g.standard_normal(N).astype(np.float32)
    A, Ah, lay = G.sketch_apply(dev(X), dev(Y), "srht", 91, [1 << 20, 1 << 21], 40)
    rows, hrows = [0, 5, 1 << 20, (1 << 21) - 1], [0, 39]
    sigma, sigma_hat = S.srht_orders(91, 22, 1 << 21, 40)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    ref = S.srht_rows(X64, Y64, 91, np.concatenate([sigma[rows], sigma_hat[hrows]]))
    bound = _srht_bound(X64, Y64, 22, U32)
    assert np.all(np.abs(A.cpu().numpy()[rows] - ref[:4]) <= bound)
    assert np.all(np.abs(Ah.cpu().numpy()[hrows] - ref[4:]) <= bound)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("N,d,m,r", [
    (20000, 19, [128, 256, 512], 120),
    (300000, 5, [1024, 2048], 24),        # ~12500 rows per S_hat bucket: 13 parts per bucket
    (60000, 3, [16384, 32768], 9000),     # S_hat counted with global atomics (r > 8192)
    (5000, 33, [2048, 4096], 40),         # many empty buckets in the largest level
    (7, 2, [2, 4], 3),                    # tiny
    (40000, 40, [64, 512, 4096], 100),    # levels 8x apart, folded in one pass
    (70000, 7, [16, 16384], 50),          # levels 1024x apart: the one-level fold
    (150000, 36, [64 << k for k in range(11)], 200),  # 11 levels: two multi-level passes
])
def test_countsketch_parity(G, dtype, N, d, m, r):
    g = np.random.default_rng(N + d)
    X = g.standard_normal((N, d)).astype(dtype)
    Y = g.standard_normal(N).astype(dtype)
    A, Ah, lay = G.sketch_apply(dev(X), dev(Y), "countsketch", 55, m, r)
    ref = S.countsketch(X.astype(np.float64), Y.astype(np.float64), 55, m, r)
    u = U64 if dtype == np.float64 else U32
    W = np.abs(S.joint(X.astype(np.float64), Y.astype(np.float64)))
    colsum = W.sum(axis=0)[None, :]
    # every bucket sums at most N terms in some order
    assert np.all(np.abs(A.cpu().numpy() - ref["A"]) <= 4 * u * colsum + 1e-300)
    assert np.all(np.abs(Ah.cpu().numpy() - ref["Ahat"]) <= 4 * u * colsum + 1e-300)
    assert lay["offset"] == ref["offset"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_gaussian_sketch_parity(G, dtype):
    N, d = 3000, 9
    g = np.random.default_rng(4)
    X = g.standard_normal((N, d)).astype(dtype)
    Y = g.standard_normal(N).astype(dtype)
    m, r = [16, 64], 40
    A, Ah, lay = G.sketch_apply(dev(X), dev(Y), "gaussian", 66, m, r)
    ref = S.gaussian(X.astype(np.float64), Y.astype(np.float64), 66, m, r)
    W = np.abs(S.joint(X.astype(np.float64), Y.astype(np.float64)))
    # G entries agree to ~2e-6 (FP32 Box-Muller); accumulation adds u_T per term
    tol = (4e-6 + 4 * N * (U64 if dtype == np.float64 else U32)) * 5 * W.sum(axis=0)[None, :]
    assert np.all(np.abs(A.cpu().numpy() - ref["A"]) <= tol)
    assert np.all(np.abs(Ah.cpu().numpy() - ref["Ahat"]) <= tol)


@pytest.mark.parametrize("N,d", [(3000, 37), (2500, 200), (1500, 520), (1200, 575), (1200, 576),
                                 (1500, 700), (1100, 1024)])
def test_gaussian_sketch_bf16_mfma_parity(G, N, d):
    # BF16 operands (G and [X|Y] rounded to nearest even), FP32 accumulation on
    # the matrix cores; compared with the oracle on the same rounded operands.
    # Staged tiles hold the 32-column tiles with data: 64 columns at d = 37,
    # every column in one block up to d = 575, two column blocks from d = 576
    # (576 + 32 columns), at d = 700 (576 + 128) and at d = 1024 (576 + 480)
    g = np.random.default_rng(6 + d)
    X = g.standard_normal((N, d)).astype(np.float32)
    Y = g.standard_normal(N).astype(np.float32)
    m, r = [32, 200], max(130, d + 40)
    A, Ah, lay = G.sketch_apply(dev(X), dev(Y), "gaussian", 88, m, r, bf16=True)
    Xb = S.round_to(X, "bf16")
    Yb = S.round_to(Y, "bf16")
    ref = S.gaussian(Xb, Yb, 88, m, r, g_round="bf16")
    W = np.abs(S.joint(Xb, Yb))
    for out, stream, rows in ((A, R.STREAM_G, 200), (Ah, R.STREAM_GHAT, r)):
        Gabs = np.abs(R.gaussian_block(88, stream, np.arange(rows), np.arange(N)))
        bound = Gabs @ W
        # FP32 accumulation (N terms) plus rare one-ulp BF16 flips of G entries
        # whose FP32 and FP64 Box-Muller values straddle a rounding boundary
        tol = (N * U32 + 2.0 ** -7 * 0.01) * bound + 1e-6
        want = ref["A"] if stream == R.STREAM_G else ref["Ahat"]
        assert np.all(np.abs(out.cpu().numpy() - want) <= tol)


# ---------------------------------------------------------------------------
# factorization
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("method", ["chol", "qr"])
@pytest.mark.parametrize("rows,d,kappa", [(192, 32, 1e2), (1536, 256, 1e4), (700, 100, 1e3),
                                          (3072, 512, 1e3)])
def test_factor_parity(G, method, rows, d, kappa):
    g = np.random.default_rng(rows + d)
    A = g.standard_normal((rows, d)) * np.logspace(0, -np.log10(kappa), d)[None, :]
    scale = 1.0 / rows
    R, M = G.factor(dev(A), d, scale, method)
    Rref = O.qr_r(np.sqrt(scale) * A)
    Rg = R.cpu().numpy()
    assert np.allclose(np.tril(Rg, -1), 0)
    assert np.all(np.diag(Rg) > 0)
    tol = (kappa ** 2 if method == "chol" else kappa) * 200 * d * U64
    assert np.linalg.norm(Rg - Rref) / np.linalg.norm(Rref) < tol
    H = Rref.T @ Rref
    Mg = M.cpu().numpy()
    assert np.linalg.norm(Mg @ H - np.eye(d)) < kappa ** 2 * 1e3 * d * U64


@pytest.mark.parametrize("rows,d,kappa", [(1536, 64, 1e8), (3072, 128, 1e12)])
def test_factor_qr_ill_conditioned(G, rows, d, kappa):
    # the Gram matrix has condition number kappa^2 (up to 1e24): only the
    # shifted CholeskyQR3 route can factor it.  A = Z diag(s) has R = R_Z diag(s),
    # so R is compared with Householder's after removing the column scale
    g = np.random.default_rng(rows + d)
    s = np.logspace(0, -np.log10(kappa), d)
    A = g.standard_normal((rows, d)) * s[None, :]
    R, _ = G.factor(dev(A), d, 1.0 / rows, "qr")
    Rref = O.qr_r(np.sqrt(1.0 / rows) * A)
    Rg = R.cpu().numpy()
    assert np.all(np.diag(Rg) > 0)
    err = np.linalg.norm((Rg - Rref) / s[None, :]) / np.linalg.norm(Rref / s[None, :])
    assert err < 1e3 * d * U64


def test_solve_qr_route_reaches_ls_error_at_kappa_1e8(G):
    # the paper's recipe X = G D with kappa = 1e8 and sigma^2 = 1e-8: the
    # prediction error reaches the LS error sigma^2 d (Sec. 5)
    from slse_inputs import paper_problem

    prob = paper_problem(1 << 15, 32, 1e8, 1e-8)
    m = G.paper_schedule(prob.n, prob.d)
    params = G.Params(kind="srht", seed=21, m=m, a=[2] * len(m), r=6 * 32, s_max=60, factor="qr")
    beta, info = G.solve(dev(prob.X), dev(prob.Y), params)
    assert info["status"] == "SLSE_OK"
    bhat, _, _ = O.ols_refined(prob.X, prob.Y)
    d_gpu = np.sum((prob.X @ (beta.cpu().numpy() - prob.beta_true)) ** 2)
    d_ls = np.sum((prob.X @ (bhat - prob.beta_true)) ** 2)
    assert abs(d_gpu / d_ls - 1) < 1e-3


@pytest.mark.parametrize("variant", ["countsketch", "auto_a", "stage2_only", "tuning"])
def test_schedule_variants_reach_ls_error(G, variant):
    # the paper's recipe (kappa = 1e4, sigma^2 = 1e-8): CountSketch levels, a_i
    # from the lower bound of Thm lowerBoundai, stage 2 alone (M-IHS) and a
    # tuning-style schedule all reach the LS error of the OLS estimator
    from slse_inputs import paper_problem

    prob = paper_problem(1 << 15, 32, 1e4, 1e-8)
    d = prob.d
    m = G.paper_schedule(prob.n, d)
    kw = dict(kind="srht", m=m, a=[2] * len(m))
    if variant == "countsketch":
        kw = dict(kind="countsketch", m=m, a=[2] * len(m))
    elif variant == "auto_a":
        kw = dict(kind="srht", m=m, a=G.auto_a(m, d, 0.5, a1=2))
    elif variant == "stage2_only":
        kw = dict(kind="srht", m=[m[0]], a=[0])
    elif variant == "tuning":
        kw = dict(kind="srht", m=[512, 1024, 2048, 8192], a=[3] * 4)
    params = G.Params(seed=31, r=6 * d, s_max=60, **kw)
    beta, info = G.solve(dev(prob.X), dev(prob.Y), params)
    assert info["status"] == "SLSE_OK"
    bhat, _, _ = O.ols_refined(prob.X, prob.Y)
    d_gpu = np.sum((prob.X @ (beta.cpu().numpy() - prob.beta_true)) ** 2)
    d_ls = np.sum((prob.X @ (bhat - prob.beta_true)) ** 2)
    assert abs(d_gpu / d_ls - 1) < 1e-6
    assert 0.2 < d_ls / (1e-8 * d) < 3.0  # chi-square with d degrees of freedom


def test_factor_singular_reports_esingular(G):
    from paper_2509_06856_amd import _lib

    A = np.random.default_rng(0).standard_normal((64, 8))
    A[:, 3] = 0.0
    with pytest.raises(_lib.SlseError) as e:
        G.factor(dev(A), 8, 1.0, "chol")
    assert e.value.status == _lib.SLSE_ESINGULAR


# ---------------------------------------------------------------------------
# whole solve
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["srht", "countsketch", "gaussian"])
def test_solve_trajectory_matches_oracle(G, kind):
    prob = make_problem("plain_small")
    m = [64, 128, 256, 512, 1024]
    a = [2] * 5
    params = G.Params(kind=kind, seed=1001, m=m, a=a, r=192, s_max=30)
    beta, info, traj, sur = G.solve(dev(prob.X), dev(prob.Y), params, record=True)
    ref_beta, ref_traj, _ = OS.slse_frs(prob.X, prob.Y, 1001, kind, m, a, 192, s=30)
    tg = traj.cpu().numpy()
    # Gaussian sketch entries agree to FP32 Box-Muller accuracy only
    tol = 1e-12 if kind != "gaussian" else 1e-5
    for t in range(len(ref_traj)):
        den = max(np.linalg.norm(ref_traj[t]), 1e-300)
        assert np.linalg.norm(tg[t] - ref_traj[t]) / den <= tol, t
    bstar, _, _ = O.ols_refined(prob.X, prob.Y)
    assert OS.rel_err(beta.cpu().numpy(), bstar) < 1e-12


@pytest.mark.parametrize("factor", ["chol", "qr"])
def test_solve_trajectory_ragged_d(G, factor):
    # d = 70: the Gram inverse takes pivot blocks of 32, 32 and 6 rows
    prob = make_problem("plain_small", n=20000, d=70)
    m = [1024, 2048, 4096]
    params = G.Params(kind="srht", seed=77, m=m, a=[2] * 3, r=420, s_max=25, factor=factor)
    beta, info, traj, sur = G.solve(dev(prob.X), dev(prob.Y), params, record=True)
    ref_beta, ref_traj, _ = OS.slse_frs(prob.X, prob.Y, 77, "srht", m, [2] * 3, 420, s=25)
    tg = traj.cpu().numpy()
    for t in range(len(ref_traj)):
        den = max(np.linalg.norm(ref_traj[t]), 1e-300)
        assert np.linalg.norm(tg[t] - ref_traj[t]) / den <= 1e-12, t


def test_solve_graph_replays_match_eager(G):
    prob = make_problem("plain_small", n=8192, d=24)
    m = [64, 128, 256, 512]
    pe = G.Params(kind="srht", seed=3, m=m, a=[2] * 4, r=144, s_max=20)
    b_eager, _ = G.solve(dev(prob.X), dev(prob.Y), pe)
    pg = G.Params(kind="srht", seed=3, m=m, a=[2] * 4, r=144, s_max=20, use_graph=True)
    X, Y = dev(prob.X), dev(prob.Y)
    for _ in range(3):
        b_graph, _ = G.solve(X, Y, pg)
        torch.cuda.synchronize()
        assert torch.equal(b_graph, b_eager)
        _ = (X.sum() + 1).item()  # eager work between replays


def test_solve_mixed_precision_reaches_1e10(G):
    prob = make_problem("mixed", n=1 << 17, d=64)
    m = G.paper_schedule(prob.n, prob.d)
    params = G.Params(kind="srht", seed=1003, m=m, a=[2] * len(m), r=6 * 64, s_max=40,
                      precision="mixed")
    beta, info = G.solve(dev(prob.X), dev(prob.Y), params)
    bstar, _, _ = O.ols_refined(prob.X, prob.Y)
    assert OS.rel_err(beta.cpu().numpy(), bstar) < 1e-10


def test_solve_tol_stops_early_and_flags(G):
    prob = make_problem("plain_small")
    m = [64, 128, 256, 512, 1024]
    params = G.Params(kind="srht", seed=1001, m=m, a=[2] * 5, r=192, s_max=60, tol=1e-13)
    beta, info = G.solve(dev(prob.X), dev(prob.Y), params)
    assert info["status"] == "SLSE_OK"
    assert info["stage2_steps"] < 60
    bstar, _, _ = O.ols_refined(prob.X, prob.Y)
    assert OS.rel_err(beta.cpu().numpy(), bstar) < 1e-12
    params.s_max = 2
    beta, info = G.solve(dev(prob.X), dev(prob.Y), params)
    assert info["status"] == "SLSE_ENOTCONV"


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def test_backward_matches_oracle_adjoint(G):
    prob = make_problem("backward", n=16384, d=16)
    w = np.random.default_rng(2).standard_normal(16)
    m = [128, 256, 512, 1024]
    params = G.Params(kind="srht", seed=1004, m=m, a=[2] * 4, r=96, s_max=40, precision="mixed")
    X, Y = dev(prob.X), dev(prob.Y)
    beta, _ = G.solve(X, Y, params)
    dX, dY, lam = G.backward(X, Y, params, beta, dev(w), grad_dtype=torch.float64)
    rX, rY, rlam, bstar = ADJ.adjoint(prob.X, prob.Y, w)
    assert np.linalg.norm(lam.cpu().numpy() - rlam) / np.linalg.norm(rlam) < 1e-9
    assert np.linalg.norm(dX.cpu().numpy() - rX) / np.linalg.norm(rX) < 1e-6
    assert np.linalg.norm(dY.cpu().numpy() - rY) / np.linalg.norm(rY) < 1e-6


# ---------------------------------------------------------------------------
# the widest rows the library takes (d = 1024, as in the paper's d = 2^10 case)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,accum", [(np.float64, "f64"), (np.float32, "f64")])
@pytest.mark.parametrize("n,d", [(3001, 1024), (2000, 1000), (700, 1023)])
def test_fused_resid_grad_widest_rows(G, n, d, dtype, accum):
    g = np.random.default_rng(n + d)
    X = g.standard_normal((n, d)).astype(dtype)
    Y = g.standard_normal(n).astype(dtype)
    beta = g.standard_normal(d)
    gg, rn = G.fused_resid_grad(dev(X), dev(Y), dev(beta), scale=0.5, accum=accum)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    ref = 0.5 * OS.full_grad(Xd, Yd, beta)
    assert np.all(np.abs(gg.cpu().numpy() - ref) <= _grad_bound(Xd, Yd, beta, U64, 0.5))


def test_srht_widest_rows(G):
    N, d, m, r = 3000, 1024, [2048, 4096], 1100
    g = np.random.default_rng(9)
    X = g.standard_normal((N, d))
    Y = g.standard_normal(N)
    A, Ah, lay = G.sketch_apply(dev(X), dev(Y), "srht", 4243, m, r)
    ref = S.srht(X, Y, 4243, m, r)
    bound = _srht_bound(X, Y, 12, U64)
    assert np.all(np.abs(A.cpu().numpy() - ref["A"]) <= bound)
    assert np.all(np.abs(Ah.cpu().numpy() - ref["Ahat"]) <= bound)


def test_solve_trajectory_widest_rows(G):
    # d = 1024: the Gram of the 6144-row Hessian sketch inverted by Gauss-Jordan
    # (32 pivot blocks), stage-1 steps on 8192- and 16384-row prefixes
    prob = make_problem("plain_small", n=1 << 15, d=1024)
    m, r = [8192, 16384], 6144
    params = G.Params(kind="srht", seed=808, m=m, a=[2, 2], r=r, s_max=6)
    beta, info, traj, sur = G.solve(dev(prob.X), dev(prob.Y), params, record=True)
    _, otraj, oinfo = OS.slse_frs(prob.X, prob.Y, 808, "srht", m, [2, 2], r, s=6)
    tr = traj.cpu().numpy()
    for t in range(1, 11):
        assert OS.rel_err(tr[t], otraj[t]) < 1e-12, t
