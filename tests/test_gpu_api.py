"""GPU checks of the boundary's newer calls and fields against the oracle:
the per-step stop estimate, per-iterate error accounting (relative error and
the prediction error Delta_t of Sec. 5), phase times, the caller-workspace
solve, the IHS baseline, FP32-accumulated stage-2 sweeps, the adjoint's
strided right-hand side, back-to-back batched calls on a side stream, the
persistent tuning cache and checkpoint / resume of a solve.
"""
import numpy as np
import pytest
import torch

from oracle import ols as O
from oracle import slse as OS
from slse_inputs import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_06856_amd import slse

    return slse


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


M_SMALL = [64, 128, 256, 512, 1024]


@pytest.mark.parametrize("kind", ["srht", "countsketch"])
def test_stop_estimate_per_step_matches_oracle(G, kind):
    p = make_problem("plain_small")
    prm = G.Params(kind=kind, seed=1001, m=M_SMALL, a=[2] * 5, r=192, s_max=30)
    beta, info, traj, sur = G.solve(dev(p.X), dev(p.Y), prm, record=True)
    _, otraj, oinfo = OS.slse_frs(p.X, p.Y, 1001, kind, M_SMALL, [2] * 5, 192, s=30)
    s_gpu = sur.cpu().numpy()
    s_ora = np.asarray(oinfo["surrogate"])
    assert len(s_gpu) == len(s_ora) == 40
    # the iterates agree to 1e-12 relative (trajectory parity); the estimate is
    # about the relative error of beta_t, so it may move by that much in absolute
    # terms, on top of 1e-10 relative
    assert np.all(np.abs(s_gpu - s_ora) <= 1e-10 * s_ora + 2e-12), np.abs(s_gpu - s_ora).max()
    assert info["surrogate0"] == s_gpu[10] and info["surrogate_final"] == s_gpu[-1]


def test_error_accounting_matches_oracle(G):
    p = make_problem("plain_small")
    X, Y = dev(p.X), dev(p.Y)
    ref = dev(p.beta_true)
    prm = G.Params(kind="srht", seed=1001, m=M_SMALL, a=[2] * 5, r=192, s_max=25)
    beta, info, traj, sur, errs = G.solve(X, Y, prm, record=True, beta_ref=ref, pred_err=True)
    _, otraj, _ = OS.slse_frs(p.X, p.Y, 1001, "srht", M_SMALL, [2] * 5, 192, s=25)
    rel = errs["rel_err"].cpu().numpy()
    pred = errs["pred_err"].cpu().numpy()
    o_rel = np.array([OS.rel_err(b, p.beta_true) for b in otraj])
    o_pred = np.array([OS.prediction_error(p.X, b, p.beta_true) for b in otraj])
    assert rel.shape == pred.shape == (36,)
    assert np.all(np.abs(rel - o_rel) <= 1e-11)
    # Delta_t is the squared norm of X e_t, e_t = beta_t - beta: the iterates'
    # 1e-12 agreement moves it by at most 2 ||X|| 1e-12 ||beta|| sqrt(Delta_t)
    nx = np.linalg.norm(p.X, 2)
    slack = 2 * nx * 1e-12 * np.linalg.norm(p.beta_true) * np.sqrt(o_pred) + 1e-9 * o_pred
    assert np.all(np.abs(pred - o_pred) <= slack + 1e-300)
    # the last iterate is at the LS error of OLS (Sec. 5): Delta_T = Delta(beta_star)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    d_ls = OS.prediction_error(p.X, bstar, p.beta_true)
    assert abs(pred[-1] / d_ls - 1) < 1e-6


def test_phase_times_reported(G):
    p = make_problem("plain_small")
    prm = G.Params(kind="srht", seed=3, m=M_SMALL, a=[2] * 5, r=192, s_max=20)
    _, info = G.solve(dev(p.X), dev(p.Y), prm)
    parts = [info[k] for k in ("ms_sketch", "ms_factor", "ms_stage1", "ms_stage2")]
    assert all(v > 0 for v in parts)
    assert abs(sum(parts) - info["ms_total"]) <= 0.02 * info["ms_total"] + 0.02
    prm.use_graph = True
    _, info = G.solve(dev(p.X), dev(p.Y), prm)
    assert info["ms_total"] > 0 and info["ms_sketch"] == 0.0


@pytest.mark.parametrize("kind,use_graph", [("srht", False), ("countsketch", True), ("gaussian", False)])
def test_solve_in_caller_workspace_equals_solve(G, kind, use_graph):
    p = make_problem("plain_small")
    X, Y = dev(p.X), dev(p.Y)
    prm = G.Params(kind=kind, seed=17, m=M_SMALL, a=[2] * 5, r=192, s_max=15, use_graph=use_graph)
    ref, _ = G.solve(X, Y, prm)
    need = G.workspace_size(X, Y, prm)
    assert need > 0
    pool = torch.empty(need + 4096, dtype=torch.uint8, device="cuda:0")
    for off in (0, 256, 4096):
        ws = pool[off: off + need]
        for _ in range(2):
            beta, info = G.solve(X, Y, prm, ws=ws)
            assert info["status"] == "SLSE_OK"
            assert torch.equal(beta, ref)
    from paper_2509_06856_amd import _lib as L
    with pytest.raises(L.SlseError):
        G.solve(X, Y, prm, ws=pool[: need - 1])


def test_workspace_size_grows_with_the_problem(G):
    small = make_problem("plain_small", n=4096, d=16)
    big = make_problem("plain_small", n=1 << 16, d=64)
    ps = G.Params(kind="srht", seed=1, m=[128, 256], a=[2, 2], r=96, s_max=5)
    mb = OS.paper_schedule(1 << 16, 64)
    pb = G.Params(kind="srht", seed=1, m=mb, a=[2] * len(mb), r=384, s_max=5)
    n_s = G.workspace_size(dev(small.X), dev(small.Y), ps)
    n_b = G.workspace_size(dev(big.X), dev(big.Y), pb)
    # at least the sketch rows and the Hessian sketch
    assert n_s >= 8 * (256 + 96) * 17 and n_b >= 8 * ((1 << 15) + 384) * 65 and n_b > n_s


@pytest.mark.parametrize("kind", ["srht", "countsketch"])
def test_ihs_matches_oracle(G, kind):
    p = make_problem("plain_small", n=1 << 15, d=32)
    r, steps = 192, 12
    beta, traj = G.ihs(dev(p.X), dev(p.Y), kind, 400, r, steps, record=True)
    _, otraj = OS.ihs(p.X, p.Y, 400, kind, r, steps)
    tr = traj.cpu().numpy()
    assert not tr[0].any() and not otraj[0].any()  # beta_0 = 0
    for t in range(1, steps + 1):
        assert OS.rel_err(tr[t], otraj[t]) < 1e-12, t
    # refreshed sketches converge to OLS
    b60 = G.ihs(dev(p.X), dev(p.Y), kind, 400, r, 60, use_graph=True).cpu().numpy()
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    assert OS.rel_err(b60, bstar) < 1e-12


def test_fp32_accumulated_sweeps_then_fp64_reach_ols(G):
    # mixed recipe at 2^17 x 64 (kappa 1e6): 20 stage-2 sweeps accumulate in FP32
    # (they stall near kappa u32), then 30 FP64-accumulated sweeps over the same
    # FP32 data reach the OLS solution of that data
    p = make_problem("mixed", n=1 << 17, d=64)
    X, Y = dev(p.X), dev(p.Y)
    m = G.paper_schedule(1 << 17, 64)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    prm = G.Params(kind="srht", seed=1003, m=m, a=[2] * len(m), r=384, s_max=50,
                   precision="mixed", fp32_sweeps=20)
    beta, info, traj, sur = G.solve(X, Y, prm, record=True)
    assert info["status"] == "SLSE_OK"
    assert OS.rel_err(beta.cpu().numpy(), bstar) < 1e-10
    tr = traj.cpu().numpy()
    s1 = sum(prm.a)
    e20 = OS.rel_err(tr[s1 + 20], bstar)
    # the FP64 sweeps contract at the M-IHS rate from where the FP32 ones stalled
    assert e20 > 1e-9
    prm0 = G.Params(**{**prm.__dict__, "fp32_sweeps": 0})
    beta0, _ = G.solve(X, Y, prm0)
    assert OS.rel_err(beta0.cpu().numpy(), bstar) < 1e-10


def test_backward_reads_a_strided_right_hand_side(G):
    p = make_problem("backward", n=8192, d=16)
    X, Y = dev(p.X), dev(p.Y)
    m = [256, 512, 1024, 2048]
    prm = G.Params(kind="srht", seed=5, m=m, a=[2] * 4, r=96, s_max=30, precision="mixed")
    beta, _ = G.solve(X, Y, prm)
    base = torch.from_numpy(np.random.default_rng(3).standard_normal(32)).to("cuda:0")
    w_strided = base[::2]
    dX1, dY1, l1 = G.backward(X, Y, prm, beta, w_strided)
    dX2, dY2, l2 = G.backward(X, Y, prm, beta, w_strided.contiguous())
    assert torch.equal(l1, l2) and torch.equal(dX1, dX2) and torch.equal(dY1, dY2)
    w0 = torch.full((1,), 0.75, dtype=torch.float64, device="cuda:0").expand(16)
    assert w0.stride(0) == 0
    _, _, l3 = G.backward(X, Y, prm, beta, w0)
    _, _, l4 = G.backward(X, Y, prm, beta, w0.contiguous())
    assert torch.equal(l3, l4)


def test_batched_calls_back_to_back_on_a_side_stream(G):
    # two different batches on a non-blocking stream without reports: the second
    # call rewrites the shared descriptor tables only after the first graph ran
    def batch(shapes, seed0):
        Xs, Ys, ps, singles = [], [], [], []
        for k, (n, d) in enumerate(shapes):
            p = make_problem("plain_small", n=n, d=d, seed=seed0 + k)
            m = G.paper_schedule(n, d)
            prm = G.Params(kind="srht", seed=seed0 + k, m=m, a=[2] * len(m), r=6 * d, s_max=10)
            Xs.append(dev(p.X))
            Ys.append(dev(p.Y))
            ps.append(prm)
            singles.append(G.solve(Xs[-1], Ys[-1], prm)[0].cpu().numpy())
        return Xs, Ys, ps, singles

    A = batch([(6000, 16), (11000, 8), (40000, 40)], 50)
    B = batch([(5000, 12), (9000, 24), (3000, 8), (20000, 16)], 70)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        outs = []
        for _ in range(3):
            for Xs, Ys, ps, _ in (A, B):
                betas, _ = G.solve_batched(Xs, Ys, ps, report=False)
                outs.append(betas)
    s.synchronize()
    for i, betas in enumerate(outs):
        singles = (A, B)[i % 2][3]
        for b, ref in zip(betas, singles):
            assert OS.rel_err(b.cpu().numpy(), ref) < 1e-13, i


def test_tuned_launch_shapes_persist_across_contexts(G, tmp_path):
    p = make_problem("plain_small", n=1 << 15, d=64)
    X, Y = dev(p.X), dev(p.Y)
    m = G.paper_schedule(1 << 15, 64)
    prm = G.Params(kind="srht", seed=21, m=m, a=[2] * len(m), r=384, s_max=8)
    c1 = G.Context(0)
    b1, _ = G.solve(X, Y, prm, ctx=c1)
    path = tmp_path / "tune.txt"
    c1.save_tuning(path)
    lines = path.read_text().splitlines()
    assert lines[0].startswith("libslse-tuning 1 gfx") and len(lines) > 1
    c2 = G.Context(0)
    assert c2.load_tuning(path) == len(lines) - 1
    b2, _ = G.solve(X, Y, prm, ctx=c2)
    assert torch.equal(b1, b2)  # same shapes, same kernels: the same result
    other = tmp_path / "other.txt"
    other.write_text("libslse-tuning 1 gfx000/1\n" + "\n".join(lines[1:]) + "\n")
    assert G.Context(0).load_tuning(other) == 0
    from paper_2509_06856_amd import _lib as L
    bad = tmp_path / "bad.txt"
    bad.write_text("something else\n")
    with pytest.raises(L.SlseError):
        c2.load_tuning(bad)
    c1.close()
    c2.close()


@pytest.mark.parametrize("kind", ["srht", "countsketch", "gaussian"])
@pytest.mark.parametrize("reset", [False, True])
@pytest.mark.parametrize("use_graph", [False, True])
def test_checkpoint_resume_retraces_the_solve(G, kind, reset, use_graph):
    # a solve stopped after k steps and resumed from its (beta_{k-1}, beta_k)
    # retraces the uninterrupted solve bit for bit (the sketch is recomputed
    # from the seed; the launch shapes and reduction orders are the same):
    # mid-subproblem, at a subproblem boundary, at the start of stage 2,
    # inside stage 2 and at the end
    p = make_problem("plain_small", n=1 << 14, d=32)
    X, Y = dev(p.X), dev(p.Y)
    prm = G.Params(kind=kind, seed=77, m=[256, 512, 1024], a=[2, 3, 2], r=192, s_max=12,
                   momentum_reset=reset, use_graph=use_graph)
    T = sum(prm.a) + prm.s_max
    beta, info, traj, sur = G.solve(X, Y, prm, record=True)
    assert info["stage1_steps"] == 7 and info["stage2_steps"] == 12
    for k in [3, 5, 7, 11, T]:  # stop_step = 0 means T
        st = torch.empty((2, 32), dtype=torch.float64, device="cuda:0")
        _, ip = G.solve(X, Y, prm, stop_step=k, state_out=st)
        assert ip["stage1_steps"] == min(k, 7) and ip["stage2_steps"] == max(0, k - 7)
        assert torch.equal(st[1], traj[k]), k
        assert torch.equal(st[0], traj[k - 1]), k
        b2, ir, traj2, sur2 = G.solve(X, Y, prm, record=True, start_step=k, beta0=st[1],
                                      beta_prev=st[0])
        assert ir["stage1_steps"] == max(0, 7 - k) and ir["stage2_steps"] == min(12, T - k)
        assert torch.equal(b2, beta), k
        assert torch.equal(traj2[k:], traj[k:]), k
        if k < T:
            assert torch.equal(sur2[k:T], sur[k:T]), k
    # the oracle's state at a checkpoint is the same iterate (Gaussian sketch
    # entries agree to FP32 Box-Muller accuracy only)
    _, otraj, _ = OS.slse_frs(p.X, p.Y, 77, kind, prm.m, prm.a, 192, 12, momentum_reset=reset)
    assert OS.rel_err(traj[5].cpu().numpy(), otraj[5]) < (1e-5 if kind == "gaussian" else 1e-12)


def test_checkpoint_fields_are_checked(G):
    p = make_problem("plain_small", n=4096, d=16)
    X, Y = dev(p.X), dev(p.Y)
    prm = G.Params(kind="srht", seed=3, m=[128, 256], a=[2, 2], r=96, s_max=4)
    for kw in (dict(start_step=9), dict(stop_step=9), dict(start_step=5, stop_step=3),
               dict(start_step=-1)):
        with pytest.raises(Exception):
            G.solve(X, Y, prm, **kw)
    beta, _ = G.solve(X, Y, prm, start_step=8)  # nothing left to run: beta_8 = beta0 = 0
    assert not beta.cpu().numpy().any()


@pytest.mark.parametrize("kind,N,r", [("srht", 20000, 300), ("gaussian", 20000, 300),
                                      ("countsketch", 20000, 300),
                                      ("countsketch", 300000, 24),    # ~12500 rows a bucket, in parts
                                      ("countsketch", 60000, 9000)])  # the fallback past 8192 buckets
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sketches_are_bit_reproducible(G, kind, N, r, dtype):
    # the same call twice gives the same bits: every reduction runs in a fixed
    # order (the CountSketch bucket lists are in row order)
    g = np.random.default_rng(5)
    d = 16
    X = dev(g.standard_normal((N, d)).astype(dtype))
    Y = dev(g.standard_normal(N).astype(dtype))
    m = [256, 512, 1024, 4096]
    bf16 = kind == "gaussian" and dtype == np.float32
    A1, H1, _ = G.sketch_apply(X, Y, kind, 21, m, r, bf16=bf16)
    A2, H2, _ = G.sketch_apply(X, Y, kind, 21, m, r, bf16=bf16)
    assert torch.equal(A1, A2) and torch.equal(H1, H2)


@pytest.mark.parametrize("N,m", [(20000, [256, 512, 1024, 2048]),       # one digit
                                 (70001, [1024, 4096, 16384, 32768]),   # two digits, ragged N
                                 (1 << 20, [4096, 1 << 17, 1 << 18, 1 << 19])])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_countsketch_sorted_lists_match_sorted_atomic_lists(G, N, m, dtype, monkeypatch):
    # the largest level's lists by the counting sort and by atomic slot claims
    # sorted afterwards hold the same rows in the same (row) order, so both
    # routes give the same sketch bit for bit
    g = np.random.default_rng(11)
    d = 24
    X = dev(g.standard_normal((N, d)).astype(dtype))
    Y = dev(g.standard_normal(N).astype(dtype))
    monkeypatch.setenv("SLSE_CS_SORT", "1")
    A1, H1, _ = G.sketch_apply(X, Y, "countsketch", 8, m, 200)
    monkeypatch.setenv("SLSE_CS_SORT", "0")
    A2, H2, _ = G.sketch_apply(X, Y, "countsketch", 8, m, 200)
    assert torch.equal(A1, A2) and torch.equal(H1, H2)


@pytest.mark.parametrize("N,d,dtype", [(1 << 13, 64, np.float32), (9000, 32, np.float32),
                                       (1 << 13, 48, np.float64), (1 << 12, 16, np.float64)])
def test_srht_own_y_passes_match_the_shared_tile(G, N, d, dtype, monkeypatch):
    # when d fills whole column tiles, Y is transformed on its own (one-column
    # passes); every column's butterflies are the same either way, so the
    # sketch must not change by a bit
    g = np.random.default_rng(13)
    X = dev(g.standard_normal((N, d)).astype(dtype))
    Y = dev(g.standard_normal(N).astype(dtype))
    m = [128, 256, 1024]
    monkeypatch.setenv("SLSE_SRHT_SPLIT_Y", "1")
    A1, H1, _ = G.sketch_apply(X, Y, "srht", 4, m, 3 * d)
    # Y gathered through P in its own first pass instead of with the index maps
    monkeypatch.setenv("SLSE_SRHT_Y_PREGATHER", "0")
    A3, H3, _ = G.sketch_apply(X, Y, "srht", 4, m, 3 * d)
    monkeypatch.setenv("SLSE_SRHT_Y_PREGATHER", "1")
    monkeypatch.setenv("SLSE_SRHT_SPLIT_Y", "0")
    A2, H2, _ = G.sketch_apply(X, Y, "srht", 4, m, 3 * d)
    assert torch.equal(A1, A2) and torch.equal(H1, H2)
    assert torch.equal(A1, A3) and torch.equal(H1, H3)
