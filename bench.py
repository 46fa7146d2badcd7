#!/usr/bin/env python
"""SLSE-FRS on one MI355X: seconds to 1e-10 relative error against the FP64 OLS
solution, the fused residual-gradient kernel's HBM bandwidth, and the
mixed-precision form against the plain FP64 form.

One step = one whole solve (sketch of [X|Y], factor of the Hessian sketch,
stage-1 steps on the nested sketches, stage-2 full-data steps) on data already
resident in HBM, replayed from a captured hipGraph.  The number of stage-2
steps is the smallest that reaches the tolerance, found by a calibration solve
that records every iterate and compares it with the stored oracle solution;
the timed solves use that count and their result is checked again.

    python bench.py [--steps K] [--warmup W] [--workload mixed|illcond]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "seconds to 1e-10 rel. error vs FP64 OLS; resid-grad HBM GB/s; mixed vs FP64"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_reference(name):
    path = os.path.join(ROOT, "tests", "golden", f"ref_{name}.json")
    with open(path) as f:
        return json.load(f)


# the residual-gradient kernel and the device helpers it uses
KERNEL_SOURCES = ("k_resid_grad.hip", "common.hpp")


def counted_traffic(name):
    """HBM bytes per residual-gradient launch from the committed counter runs,
    or None when they were not taken on this workload or the kernel source has
    changed since."""
    if name != "mixed":
        return None
    path = os.path.join(ROOT, "profiles", "resid_grad_f32_4194304x512_counters.md")
    csrc = os.path.join(ROOT, "paper_2509_06856_amd", "csrc")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if ": " in line and not line.startswith(("-", "|", "#")))
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(csrc, f), "rb").read())
        digest = h.hexdigest()
    except OSError:
        return None
    if fields.get("kernel sources sha256", "").strip() != digest:
        return None
    return int(fields["traffic_bytes_per_launch"])


def rel_err(b, ref):
    return float(np.linalg.norm(b - ref) / np.linalg.norm(ref))


def calibrate(G, torch, X, Y, params, beta_star, tol, s_cap):
    """Smallest stage-2 step count whose iterate meets tol (from one recorded solve)."""
    params.s_max = s_cap
    params.use_graph = False
    beta, info, traj, sur = G.solve(X, Y, params, record=True)
    tr = traj.cpu().numpy()
    s1 = sum(params.a)
    errs = [rel_err(tr[s1 + s], beta_star) for s in range(s_cap + 1)]
    for s, e in enumerate(errs):
        if e <= tol:
            return s, errs
    return None, errs


def time_solves(G, torch, X, Y, params, steps, warmup):
    params.use_graph = True
    beta = None
    for _ in range(warmup):
        beta, _ = G.solve(X, Y, params, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        beta, _ = G.solve(X, Y, params, report=False)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, beta


def time_resid_grad(G, torch, X, Y, beta, reps=20):
    """Average device time of one fused residual-gradient launch (HIP events)."""
    for _ in range(3):
        G.fused_resid_grad(X, Y, beta)
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        G.fused_resid_grad(X, Y, beta)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def time_calls(torch, fn, reps=3):
    """Average device seconds of fn() over reps calls (HIP events, current stream)."""
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def measure_kernels(G, torch, X, Y, m, r, seed):
    """Sketch kernels on the workload's own data (each sketch call is one
    slse_sketch_apply, index maps included), and the two reference streams they
    are stated against: a plain streaming read of X and a plain copy of X."""
    N, d = X.shape
    row = (d + 1) * X.element_size()
    out = {}
    xbytes = X.numel() * X.element_size()
    sink = torch.empty(1 << 16, dtype=torch.int32, device=X.device)
    # the ceilings are what a bare stream reaches at best: the fastest of
    # three rounds of 20 launches each
    t = min(time_calls(torch, lambda: G.debug_bandwidth(0, X, sink), reps=20) for _ in range(3))
    out["stream_read_GBs"] = xbytes / t / 1e9
    Z = torch.empty_like(X)
    t = min(time_calls(torch, lambda: G.debug_bandwidth(1, X, Z), reps=20) for _ in range(3))
    out["stream_copy_GBs"] = 2 * xbytes / t / 1e9
    del Z
    torch.cuda.empty_cache()
    t = time_calls(torch, lambda: G.sketch_apply(X, Y, "srht", seed, [m[-1]], r))
    alg = (N + m[-1] + r) * row
    out["srht"] = {"ms": t * 1e3, "GBs": alg / t / 1e9, "frac_of_peak": alg / t / 1e9 / HBM_PEAK_GBS,
                   "algorithmic_bytes": alg,
                   "note": "read [X|Y] once, write m_K + r sampled rows; two passes over a padded workspace"}
    t = time_calls(torch, lambda: G.sketch_apply(X, Y, "countsketch", seed, m, r))
    alg = (N + sum(m) + r) * row
    out["countsketch"] = {"ms": t * 1e3, "GBs": alg / t / 1e9,
                          "frac_of_peak": alg / t / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": alg,
                          "note": "read [X|Y] once, write every level and the r Hessian buckets"}
    for k in ("srht", "countsketch"):
        # both read and write: stated against the plain copy's read + write rate
        out[k]["frac_of_stream_copy"] = out[k]["GBs"] / out["stream_copy_GBs"]
    if X.dtype == torch.float32:
        # the Gaussian sketch is a dense contraction: report it against the BF16 MFMA peak
        mg = [r]
        t = time_calls(torch, lambda: G.sketch_apply(X, Y, "gaussian", seed, mg, r, bf16=True), reps=2)
        flops = 2.0 * (mg[-1] + r) * N * (d + 1)
        # the floor the VALU work sets: the same entries of G generated alone
        sink = torch.empty(256 * 1024, dtype=torch.int32, device=X.device)
        t_gen = time_calls(torch, lambda: [G.debug_gaussian_generate(seed, st, rows, N, 1024, sink=sink)
                                           for st, rows in ((7, mg[-1]), (8, r))], reps=2)
        out["gaussian_bf16"] = {"ms": t * 1e3, "TFLOPs": flops / t / 1e12,
                                "frac_of_peak": flops / t / 1e12 / BF16_PEAK_TFLOPS,
                                "flops": flops, "sketch_rows": mg[-1] + r,
                                "valu_floor_ms": t_gen * 1e3,
                                "time_over_valu_floor": t / t_gen,
                                "note": "G generated on the fly (Philox + Box-Muller), BF16 MFMA, FP32 "
                                        "accumulation; valu_floor_ms: the same entries of G generated "
                                        "alone (slse_debug_gaussian_generate)"}
    return out


def cpu_baseline(name, d, seed, tol, n_sample, s_hint):
    """The oracle on a same-recipe sample of n_sample rows, on every core this
    process may use (BLAS threads set to that count): O1 (Householder-QR OLS
    with refinement) and O2 (the seeded SLSE-FRS iteration, paper schedule) to
    tol against the sample's own OLS solution.  The stage-2 count is the
    oracle's own, found by an untimed run that records every iterate."""
    from threadpoolctl import threadpool_limits

    from oracle import ols as O
    from oracle import slse as OS
    from slse_inputs import make_problem

    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(cores):
        p = make_problem(name, n=n_sample)
        t0 = time.perf_counter()
        bstar, _, _ = O.ols_refined(p.X, p.Y)
        t_o1 = time.perf_counter() - t0
        m = OS.paper_schedule(n_sample, d)
        s1 = 2 * len(m)
        _, traj, _ = OS.slse_frs(p.X, p.Y, seed, "srht", m, [2] * len(m), 6 * d, s=s_hint + 15)
        s_cpu = next((s for s in range(s_hint + 16) if rel_err(traj[s1 + s], bstar) <= tol), None)
        if s_cpu is None:
            return None
        t0 = time.perf_counter()
        beta, _, _ = OS.slse_frs(p.X, p.Y, seed, "srht", m, [2] * len(m), 6 * d, s=s_cpu)
        t_o2 = time.perf_counter() - t0
    return dict(t_o1=t_o1, t_o2=t_o2, s=s_cpu, err=rel_err(beta, bstar), cores=cores)


def cpu_single_core_small(tol=1e-12):
    """The oracle on the small FP64 problem (16384 x 32) on one core: O1, and O2
    to tol against O1 with the problem's own schedule (m = 2d..32d, r = 6d)."""
    from threadpoolctl import threadpool_limits

    from oracle import ols as O
    from oracle import slse as OS
    from slse_inputs import make_problem, sketch_seed

    with threadpool_limits(1):
        p = make_problem("plain_small")
        t0 = time.perf_counter()
        bstar, _, _ = O.ols_refined(p.X, p.Y)
        t_o1 = time.perf_counter() - t0
        m = [64, 128, 256, 512, 1024]
        seed = sketch_seed("plain_small")
        _, traj, _ = OS.slse_frs(p.X, p.Y, seed, "srht", m, [2] * 5, 192, s=60)
        s_cpu = next((s for s in range(61) if rel_err(traj[10 + s], bstar) <= tol), 60)
        t0 = time.perf_counter()
        beta, _, _ = OS.slse_frs(p.X, p.Y, seed, "srht", m, [2] * 5, 192, s=s_cpu)
        t_o2 = time.perf_counter() - t0
    return {"workload": "plain_small: N=16384, d=32, float64", "cores": 1, "tol": tol,
            "ols_seconds": t_o1, "slse_frs_seconds": t_o2, "stage2_steps": s_cpu,
            "rel_err": rel_err(beta, bstar)}


PAPER_CASES = {
    # key: (N, d, kappa, methods) -- the problems of Sec. 5.2-5.4
    "17": (1 << 17, 64, 1e4, ("srht", "countsketch")),
    "18": (1 << 18, 64, 1e4, ("srht", "countsketch")),
    "19": (1 << 19, 64, 1e4, ("srht", "countsketch")),
    "20": (1 << 20, 64, 1e4, ("srht", "countsketch", "auto_a", "mihs_only", "ihs")),
    "20k8": (1 << 20, 64, 1e8, ("srht", "mihs_only")),
    "22": (1 << 22, 64, 1e8, ("srht", "countsketch", "tuning")),
    "20d1024": (1 << 20, 1024, 1e8, ("srht",)),
}


def paper_rows(G, torch, dev, keys):
    """The paper's own problems (Sec. 5 recipe: X = G D, D log-spaced 1..1/kappa,
    sigma^2 = 1e-8, FP64) with the schedule variants and baselines that run on
    the same kernels.  The library records the prediction error
    Delta_t = ||X (beta_t - beta)||^2 of every iterate (beta the true
    coefficients); each method is then timed, with its graph replayed, to the
    first iterate within 1% of the LS error (the smallest final Delta of the
    methods, which all reach OLS).  Returns one record per (problem, method)."""
    from slse_inputs import paper_problem

    sigma2 = 1e-8
    rows = []

    def first_within(ds, target):
        return next((t for t, v in enumerate(ds) if v <= target), None)

    for key in keys:
        N, d, kappa, methods = PAPER_CASES[key]
        t0 = time.perf_counter()
        prob = paper_problem(N, d, kappa, sigma2)
        X = torch.from_numpy(prob.X).to(dev)
        Y = torch.from_numpy(prob.Y).to(dev)
        bt = torch.from_numpy(prob.beta_true).to(dev)
        # X beta for the IHS iterates' Delta_t (fused pass with Y = X beta), formed on the host
        XB = torch.from_numpy(prob.X @ prob.beta_true).to(dev) if "ihs" in methods else None
        del prob
        log(f"paper N={N} d={d} kappa={kappa:g}: generated in {time.perf_counter() - t0:.1f}s")
        # the Gram route (Gauss-Jordan inverse) is scale-invariant for X = G D; the
        # QR route (shifted CholeskyQR3) is used at kappa = 1e8 where d allows it
        factor = "qr" if kappa > 1e6 and d <= 512 else "chol"
        m = G.paper_schedule(N, d)
        r = 6 * d
        plans = {"srht": dict(kind="srht", m=m, a=[2] * len(m)),
                 "countsketch": dict(kind="countsketch", m=m, a=[2] * len(m)),
                 "auto_a": dict(kind="srht", m=m, a=G.auto_a(m, d, 0.5, a1=2)),
                 "mihs_only": dict(kind="srht", m=[m[0]], a=[0])}
        if N == 1 << 22:
            mt = [1 << k for k in range(10, 17)] + [1 << 19]
            plans["tuning"] = dict(kind="srht", m=mt, a=[3] * len(mt))
        recs = {}
        for name in methods:
            if name == "ihs":
                continue
            prm = G.Params(seed=7000 + len(rows) + len(recs), r=r, s_max=60, factor=factor,
                           **plans[name])
            _, info, errs = G.solve(X, Y, prm, beta_ref=bt, pred_err=True)
            recs[name] = (prm, errs["pred_err"].cpu().numpy(), info["status"])
        d_ls = min(ds[-1] for _, ds, _ in recs.values())
        for name in methods:
            if name == "ihs":
                continue
            prm, ds, status = recs[name]
            s1 = sum(prm.a)
            hit = first_within(ds, 1.01 * d_ls)
            rec = {"N": N, "d": d, "kappa": kappa, "method": name, "factor": factor,
                   "status": status, "ls_error_over_sigma2d": d_ls / (sigma2 * d),
                   "delta_T_over_ls": float(ds[-1] / d_ls), "iterations_to_1pct": hit}
            if hit is not None:
                prm.s_max = max(0, hit - s1)
                t_s, _ = time_solves(G, torch, X, Y, prm, 5, 1)
                rec["seconds_to_1pct"] = t_s
            rows.append(rec)
            log(f"  {name}: Delta_T/LS {rec['delta_T_over_ls']:.4f}, iterations {hit}, "
                f"{rec.get('seconds_to_1pct', float('nan')) * 1e3:.2f} ms")
        if "ihs" in methods:
            # IHS with a fresh Hessian sketch every step (slse_ihs, mu = 1, eta = 0);
            # Delta_t from the fused pass with Y = X beta
            _, traj = G.ihs(X, Y, "srht", 9000, r, 40, record=True, factor=factor)
            ds = [G.fused_resid_grad(X, XB, traj[t])[1].item() for t in range(traj.shape[0])]
            hit = first_within(ds, 1.01 * d_ls)
            rec = {"N": N, "d": d, "kappa": kappa, "method": "ihs_refreshed_hessian",
                   "factor": factor, "ls_error_over_sigma2d": d_ls / (sigma2 * d),
                   "delta_T_over_ls": ds[-1] / d_ls, "iterations_to_1pct": hit}
            if hit is not None:
                G.ihs(X, Y, "srht", 9000, r, hit, factor=factor, use_graph=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    G.ihs(X, Y, "srht", 9000, r, hit, factor=factor, use_graph=True)
                torch.cuda.synchronize()
                rec["seconds_to_1pct"] = (time.perf_counter() - t0) / 3
            rows.append(rec)
            log(f"  ihs_refreshed_hessian: Delta/LS {rec['delta_T_over_ls']:.4f}, iterations "
                f"{rec['iterations_to_1pct']}, {rec.get('seconds_to_1pct', float('nan')) * 1e3:.2f} ms")
            del XB
        del X, Y
        torch.cuda.empty_cache()
    return rows


def bench_paper(args, G, torch, dev):
    """`--workload paper`: the table of paper_rows as its own JSON line."""
    keys = args.paper_cases.split(",") if args.paper_cases else list(PAPER_CASES)
    rows = paper_rows(G, torch, dev, keys)
    main = [r for r in rows if r["N"] == 1 << 22 and r["method"] == "srht"]
    main = main[0] if main else rows[0]
    out = {
        "metric": METRIC, "value": main.get("seconds_to_1pct"), "unit": "s", "n_gpus": 1,
        "steps": 5, "warmup": 1, "ms_per_step": (main.get("seconds_to_1pct") or 0) * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "paper: X = G D, sigma^2 = 1e-8, the problems of Sec. 5.2-5.4 "
                               "(d = 64 at N = 2^17..2^20, kappa 1e4; 2^20 and 2^22 at kappa 1e8; "
                               "d = 1024 at 2^20, kappa 1e8); time to within 1% of the LS error",
                   "results": rows},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_backward(args, G, torch, dev):
    """Adjoint of beta_hat for L = w^T beta_hat on the backward workload (2^20 x 256,
    float32): lambda by the sketch-preconditioned iteration, then the fused
    rank-2 pass; errors against the stored FP64 oracle lambda and beta_star."""
    from slse_inputs import fingerprint, make_problem, sketch_seed

    ref = load_reference("backward")
    prob = make_problem("backward")
    if fingerprint(prob.X, prob.Y) != ref["fingerprint"]:
        print("regenerated backward data differ from the stored reference", file=sys.stderr)
        sys.exit(3)
    N, d = prob.n, prob.d
    X = torch.from_numpy(prob.X).to(dev)
    Y = torch.from_numpy(prob.Y).to(dev)
    bstar = np.asarray(ref["beta_star"])
    lam_ref = np.asarray(ref["lambda"])
    w = torch.from_numpy(np.asarray(ref["w"])).to(dev)
    m = G.paper_schedule(N, d)
    params = G.Params(kind="srht", seed=sketch_seed("backward"), m=m, a=[2] * len(m), r=6 * d,
                      precision="mixed")
    if args.kernel_only:
        # the rank-2 pass (lambda_0 = M w, then one read of [X|Y] and one write
        # of [dX|dY] in float32), ten times, then a copy of X
        p0 = G.Params(**{**params.__dict__, "s_max": 0})
        b0 = torch.from_numpy(bstar).to(dev)
        for _ in range(10):
            G.backward(X, Y, p0, b0, w)
        torch.cuda.synchronize()
        log(f"rank-2 pass: 10 calls, N={N}, d={d}")
        for _ in range(3):
            Z = X.clone()
        torch.cuda.synchronize()
        log(f"copy reference: {X.numel() * X.element_size()} bytes read and written per launch")
        return
    s_star, _ = calibrate(G, torch, X, Y, params, bstar, args.tol, args.s_cap)
    if s_star is None:
        print("forward solve did not reach the tolerance", file=sys.stderr)
        sys.exit(4)
    params.s_max = s_star
    beta, _ = G.solve(X, Y, params)
    # lambda uses the same preconditioned iteration: the forward count, doubled
    # until the adjoint reaches 1e-9 against the oracle lambda
    for s_lam in (s_star, 2 * s_star, 4 * s_star):
        params.s_max = s_lam
        dX, dY, lam = G.backward(X, Y, params, beta, w, grad_dtype=torch.float64)
        e_lam = rel_err(lam.cpu().numpy(), lam_ref)
        if e_lam < 1e-9:
            break
    Xd = prob.X.astype(np.float64)
    u = Xd @ lam_ref
    r = prob.Y.astype(np.float64) - Xd @ bstar
    e_dY = float(np.linalg.norm(dY.cpu().numpy() - u) / np.linalg.norm(u))
    dXg = dX.cpu().numpy()
    ref_dX = np.outer(r, lam_ref)
    ref_dX -= np.outer(u, bstar)
    e_dX = float(np.linalg.norm(dXg - ref_dX) / np.linalg.norm(ref_dX))
    e_max = float(np.abs(dXg - ref_dX).max())
    del dX, dY, dXg, ref_dX, Xd
    log(f"adjoint: {s_lam} steps, lambda err {e_lam:.2e}, dX err {e_dX:.2e}, dY err {e_dY:.2e}")
    # timed: the production call (float32 gradients)
    t_bw = time_calls(torch, lambda: G.backward(X, Y, params, beta, w), reps=args.steps)
    # the rank-2 pass alone: lambda_0 = M w and one read of [X|Y], one write of [dX|dY]
    p0 = G.Params(**{**params.__dict__, "s_max": 0})
    t_k9 = time_calls(torch, lambda: G.backward(X, Y, p0, beta, w), reps=args.steps)
    k9_bytes = 2 * N * (d + 1) * 4
    nb = N * d * 4
    t_k = time_resid_grad(G, torch, X, None, beta)
    gbs = nb / t_k / 1e9
    log(f"backward: {t_bw * 1e3:.2f} ms; rank-2 pass {t_k9 * 1e3:.3f} ms "
        f"({k9_bytes / t_k9 / 1e9:.0f} GB/s); lambda sweep {t_k * 1e3:.3f} ms ({gbs:.0f} GB/s)")
    out = {
        "metric": METRIC, "value": t_bw, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_bw * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 storage, f64 accumulation",
        "data": "synthetic",
        "config": {"workload": f"backward: N={N}, d={d}, X iid N(0,1) float32, L = w^T beta_hat",
                   "adjoint_steps": s_lam, "lambda_rel_err": e_lam, "dX_rel_err_fro": e_dX,
                   "dX_max_abs_err": e_max, "dY_rel_err": e_dY, "forward_stage2_steps": s_star},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "resid_grad_kernel with Y = 0 (the lambda sweeps)",
                     "algorithmic_bytes": nb},
        "cpu_baseline": None,
        "kernels": {"adjoint_rank2_pass": {"ms": t_k9 * 1e3, "GBs": k9_bytes / t_k9 / 1e9,
                                           "frac_of_peak": k9_bytes / t_k9 / 1e9 / HBM_PEAK_GBS,
                                           "algorithmic_bytes": k9_bytes,
                                           "note": "s_max = 0 backward: lambda_0 = M w plus the fused pass"}},
    }
    return out


def bench_batched(args, G, torch, dev):
    """64 uneven FP32 regressions in one batched solve (one captured graph)."""
    from slse_inputs import fingerprint, make_batched

    ref = load_reference("batched")
    t0 = time.perf_counter()
    probs = make_batched()
    log(f"generated {len(probs)} problems in {time.perf_counter() - t0:.1f}s")
    for p, r in zip(probs, ref["problems"]):
        if fingerprint(p.X, p.Y) != r["fingerprint"]:
            print("regenerated batched data differ from the stored reference", file=sys.stderr)
            sys.exit(3)
    stars = [np.asarray(r["beta_star"]) for r in ref["problems"]]
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    Ys = [torch.from_numpy(p.Y).to(dev) for p in probs]
    seed0 = 1005

    def params(ss):
        out = []
        for i, p in enumerate(probs):
            m = G.paper_schedule(p.n, p.d)
            out.append(G.Params(kind="srht", seed=seed0 + 100 * i, m=m, a=[2] * len(m), r=6 * p.d,
                                s_max=ss[i], precision="mixed"))
        return out

    # each problem gets the smallest stage-2 count that reaches tol (recorded
    # single solves); heavy-tailed rows make a few problems converge slowly
    cap = max(args.s_cap, 400)
    s_each = []
    for i, p in enumerate(probs):
        prm = params([cap] * len(probs))[i]
        _, _, traj, _ = G.solve(Xs[i], Ys[i], prm, record=True)
        tr = traj.cpu().numpy()
        s1 = sum(prm.a)
        hit = next((s for s in range(cap + 1) if rel_err(tr[s1 + s], stars[i]) <= args.tol), None)
        if hit is None:
            print(f"batched: problem {i} does not reach {args.tol} in {cap} steps", file=sys.stderr)
            sys.exit(4)
        s_each.append(hit)
    log(f"calibration: stage-2 steps per problem: median {int(np.median(s_each))}, "
        f"max {max(s_each)} (problem {int(np.argmax(s_each))})")
    ps = params(s_each)
    for _ in range(args.warmup):
        G.solve_batched(Xs, Ys, ps, report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        betas, _ = G.solve_batched(Xs, Ys, ps, report=False)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    worst = max(rel_err(b.cpu().numpy(), st) for b, st in zip(betas, stars))
    if worst > args.tol:
        print(f"batched: timed solve missed the tolerance ({worst:.3e})", file=sys.stderr)
        sys.exit(5)
    rows = sum(p.n for p in probs)
    stage1_bytes = sum(2 * sum(G.paper_schedule(p.n, p.d)) * (p.d + 1) * 4 for p in probs)
    moved = sum(s_each[i] * p.n * (p.d + 1) * 4 for i, p in enumerate(probs)) + stage1_bytes
    gbs = moved / t / 1e9
    log(f"batched solve: {t * 1e3:.2f} ms for {len(probs)} problems, worst rel err {worst:.2e}")
    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_info

        from oracle import slse as OS

        sample = probs[:4]
        t1 = time.perf_counter()
        for i, p in enumerate(sample):
            m = OS.paper_schedule(p.n, p.d)
            OS.slse_frs(p.X, p.Y, seed0 + 100 * i, "srht", m, [2] * len(m), 6 * p.d, s=s_each[i])
        tc = time.perf_counter() - t1
        srows = sum(p.n * p.d for p in sample)
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        cpu = {"value": tc * sum(p.n * p.d for p in probs) / srows, "unit": "s", "cores": threads,
               "kind": "oracle",
               "sample": f"oracle SLSE-FRS on the first 4 problems ({tc:.2f}s), scaled by total N*d"}
    out = {
        "metric": METRIC, "value": t, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 storage, f64 accumulation",
        "data": "synthetic",
        "config": {"workload": f"batched: {len(probs)} problems, N_b in [2^14, 2^18], "
                               "d_b in {16..256}, Student-t(3) rows, float32",
                   "rows_total": rows, "stage2_steps_median": int(np.median(s_each)),
                   "stage2_steps_max": max(s_each), "worst_rel_err": worst,
                   "tol": args.tol},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole batched solve: algorithmic sweep bytes / solve time",
                     "algorithmic_bytes": moved},
        "cpu_baseline": cpu,
    }
    return out


def side_record(rec):
    """A workload's record as appended to the default run's line (no CPU leg)."""
    return {k: rec.get(k) for k in ("value", "unit", "ms_per_step", "dtype", "config", "roofline",
                                    "kernels") if rec.get(k) is not None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed",
                    choices=["mixed", "illcond", "batched", "backward", "paper"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--paper-cases", default="",
                    help="comma-separated keys of PAPER_CASES for --workload paper (default: all)")
    ap.add_argument("--s-cap", type=int, default=60)
    ap.add_argument("--no-f64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the paper's problems (Sec. 5), the backward and the batched workloads "
                         "that the default run appends to config")
    ap.add_argument("--no-sketches", action="store_true",
                    help="skip the sketch-kernel and device-copy measurements")
    ap.add_argument("--cpu-rows", type=int, default=1 << 18)
    ap.add_argument("--kernel-only", action="store_true",
                    help="only loop the fused residual-gradient kernel (backward: the rank-2 "
                         "adjoint pass), then a copy of X (for counter runs)")
    ap.add_argument("--gaussian-only", action="store_true",
                    help="only run three BF16 Gaussian sketch pairs (for a profiler)")
    ap.add_argument("--sketch-only", action="store_true",
                    help="only loop the SRHT and CountSketch sketches, then a copy of X "
                         "(for counter runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2509_06856_amd import slse as G
    from slse_inputs import fingerprint, make_problem, sketch_seed

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda", 0)
    name = args.workload
    if name == "batched":
        print(json.dumps(bench_batched(args, G, torch, dev)), flush=True)
        return
    if name == "backward":
        rec = bench_backward(args, G, torch, dev)
        if rec is not None:
            print(json.dumps(rec), flush=True)
        return
    if name == "paper":
        return bench_paper(args, G, torch, dev)
    ref = load_reference(name)
    beta_star = np.asarray(ref["beta_star"])

    t0 = time.perf_counter()
    prob = make_problem(name)
    log(f"generated {name} N={prob.n} d={prob.d} {prob.X.dtype} in {time.perf_counter() - t0:.1f}s")
    fp = fingerprint(prob.X, prob.Y)
    if fp != ref["fingerprint"]:
        print(f"regenerated data differ from the stored reference ({fp} != {ref['fingerprint']})",
              file=sys.stderr)
        sys.exit(3)
    N, d = prob.n, prob.d
    X = torch.from_numpy(prob.X).to(dev)
    Y = torch.from_numpy(prob.Y).to(dev)
    del prob
    mixed = X.dtype == torch.float32
    m = G.paper_schedule(N, d)
    params = G.Params(kind="srht", seed=sketch_seed(name), m=m, a=[2] * len(m), r=6 * d,
                      precision="mixed" if mixed else "f64")
    bytes_per_sweep = N * (d + 1) * X.element_size()

    if args.sketch_only:
        # three SRHT sketches (m_K + r rows), three CountSketches (every level)
        for kind, mm in (("srht", [m[-1]]), ("countsketch", m)):
            for _ in range(3):
                G.sketch_apply(X, Y, kind, params.seed, mm, 6 * d)
            torch.cuda.synchronize()
            log(f"{kind}: 3 sketches of N={N}, m_K={mm[-1]}, r={6 * d}")
        for _ in range(3):
            Z = X.clone()
        torch.cuda.synchronize()
        log(f"copy reference: {X.numel() * X.element_size()} bytes read and written per launch")
        return
    if args.gaussian_only:
        # three BF16 Gaussian sketch pairs (S and S_hat of r = 6d rows each)
        if not mixed:
            raise SystemExit("--gaussian-only needs the FP32 (mixed) workload")
        for _ in range(3):
            G.sketch_apply(X, Y, "gaussian", params.seed, [6 * d], 6 * d, bf16=True)
        # the VALU floor: the same entries of G generated alone, three times
        sink = torch.empty(256 * 1024, dtype=torch.int32, device=X.device)
        for _ in range(3):
            for st in (7, 8):
                G.debug_gaussian_generate(params.seed, st, 6 * d, N, 1024, sink=sink)
        torch.cuda.synchronize()
        log(f"gaussian_bf16: 3 sketch pairs of N={N}, {6 * d} + {6 * d} rows, then 3 generation-only "
            f"pairs")
        return
    if args.kernel_only:
        beta0 = torch.from_numpy(beta_star).to(dev)
        t_k = time_resid_grad(G, torch, X, Y, beta0, reps=50)
        log(f"resid_grad {t_k * 1e3:.3f} ms, {bytes_per_sweep / t_k / 1e9:.0f} GB/s")
        # reference for hardware byte counters: a plain device copy of X (reads and
        # writes X.numel() * element_size bytes per launch)
        for _ in range(3):
            Z = X.clone()
        torch.cuda.synchronize()
        log(f"copy reference: {X.numel() * X.element_size()} bytes read and written per launch")
        del Z
        return

    s_star, errs = calibrate(G, torch, X, Y, params, beta_star, args.tol, args.s_cap)
    log(f"calibration: stage-2 steps to {args.tol:g}: {s_star}; errors "
        + " ".join(f"{e:.1e}" for e in errs[:: max(1, len(errs) // 12)]))
    if s_star is None:
        print(f"tolerance {args.tol} not reached in {args.s_cap} stage-2 steps", file=sys.stderr)
        sys.exit(4)
    params.s_max = s_star
    t_solve, beta = time_solves(G, torch, X, Y, params, args.steps, args.warmup)
    err = rel_err(beta.cpu().numpy(), beta_star)
    log(f"{params.precision} solve: {t_solve * 1e3:.2f} ms, rel err {err:.2e}")
    if err > args.tol:
        print(f"timed solve missed the tolerance: {err:.3e}", file=sys.stderr)
        sys.exit(5)

    # the production stop: tol on the library's own estimate ||M g_t|| / ||beta_{t+1}||
    # (no oracle in the loop), with the stage-2 cap of the calibration
    prod = G.Params(**{**params.__dict__, "tol": args.tol, "s_max": args.s_cap})
    t_prod, b_prod = time_solves(G, torch, X, Y, prod, max(3, args.steps // 2), 1)
    prod.use_graph = False
    _, info_prod = G.solve(X, Y, prod)
    e_prod = rel_err(b_prod.cpu().numpy(), beta_star)
    surrogate_stop = {"seconds": t_prod, "stage2_steps": info_prod["stage2_steps"],
                      "rel_err": e_prod, "status": info_prod["status"],
                      "phase_ms": {k: info_prod[k] for k in ("ms_sketch", "ms_factor", "ms_stage1",
                                                              "ms_stage2")}}
    log(f"surrogate stop: {t_prod * 1e3:.2f} ms, {info_prod['stage2_steps']} stage-2 steps, "
        f"rel err {e_prod:.2e}; phases (ms) " + " ".join(
            f"{k[3:]} {v:.2f}" for k, v in surrogate_stop["phase_ms"].items()))

    beta_dev = torch.from_numpy(beta_star).to(dev)
    t_k = time_resid_grad(G, torch, X, Y, beta_dev)
    gbs = bytes_per_sweep / t_k / 1e9
    log(f"resid_grad: {t_k * 1e3:.3f} ms per sweep, {gbs:.0f} GB/s")

    f64 = None
    if mixed and not args.no_f64:
        X64 = X.double()
        Y64 = Y.double()
        p64 = G.Params(kind="srht", seed=params.seed, m=m, a=[2] * len(m), r=6 * d, precision="f64")
        s64, _ = calibrate(G, torch, X64, Y64, p64, beta_star, args.tol, args.s_cap)
        if s64 is not None:
            p64.s_max = s64
            t64, b64 = time_solves(G, torch, X64, Y64, p64, max(3, args.steps // 2), 1)
            e64 = rel_err(b64.cpu().numpy(), beta_star)
            t_k64 = time_resid_grad(G, torch, X64, Y64, beta_dev)
            f64 = dict(seconds=t64, stage2_steps=s64, rel_err=e64,
                       resid_grad_GBs=2 * bytes_per_sweep / t_k64 / 1e9)
            log(f"f64 solve: {t64 * 1e3:.2f} ms ({s64} stage-2 steps), rel err {e64:.2e}")
        del X64, Y64
        torch.cuda.empty_cache()

    kernels = None
    if not args.no_sketches:
        kernels = measure_kernels(G, torch, X, Y, m, 6 * d, params.seed)
        kernels["resid_grad"] = {"ms": t_k * 1e3, "GBs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
                                 "frac_of_stream_read": gbs / kernels["stream_read_GBs"]}
        log("kernels: " + ", ".join(
            f"{k} {v['ms']:.2f} ms" + (f" {v['GBs']:.0f} GB/s" if "GBs" in v else f" {v['TFLOPs']:.0f} TFLOP/s")
            for k, v in kernels.items() if isinstance(v, dict))
            + f"; stream read {kernels['stream_read_GBs']:.0f} GB/s, copy {kernels['stream_copy_GBs']:.0f} GB/s")

    cpu = None
    if not args.no_cpu:
        n_s = min(args.cpu_rows, N)
        cb = cpu_baseline(name, d, params.seed, args.tol, n_s, s_star)
        if cb is not None:
            cpu = {"value": cb["t_o2"] * N / n_s, "unit": "s", "cores": cb["cores"], "kind": "oracle",
                   "sample": (f"oracle SLSE-FRS (NumPy FP64, same recipe, paper schedule) on N={n_s} "
                              f"rows to {args.tol:g} of that sample's OLS: {cb['s']} stage-2 steps "
                              f"(the oracle's own count), {cb['t_o2']:.2f}s, rel err {cb['err']:.1e}; "
                              f"scaled by N/{n_s} to the full workload.  The OLS oracle (TSQR + "
                              f"refinement) took {cb['t_o1']:.2f}s on the sample "
                              f"(~{cb['t_o1'] * N / n_s:.0f}s scaled)"),
                   "ols_seconds_sample": cb["t_o1"], "slse_frs_seconds_sample": cb["t_o2"],
                   "single_core_small": cpu_single_core_small()}
            log(f"cpu oracle sample: O2 {cb['t_o2']:.2f}s ({cb['s']} steps), O1 {cb['t_o1']:.2f}s "
                f"on {n_s} rows ({cb['cores']} cores), err {cb['err']:.1e}")

    paper = backward = batched = None
    if not args.no_others and name == "mixed":
        # the paper's problems, the backward and the batched workloads on the
        # same library (not part of the metric; their own CPU legs skipped):
        # the mixed workload's data are freed first
        del X, Y, beta_dev
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        paper = paper_rows(G, torch, dev, list(PAPER_CASES))
        log(f"paper problems: {len(paper)} results in {time.perf_counter() - t0:.1f}s")
        side = argparse.Namespace(**{**vars(args), "no_cpu": True, "kernel_only": False})

        def run_side(fn):
            # a side workload that misses its own checks is recorded as such;
            # the main line is still printed
            try:
                return side_record(fn(side, G, torch, dev))
            except SystemExit as e:
                return {"error": f"exited with status {e.code}"}
            except Exception as e:  # a library error: recorded, the main line still printed
                print(f"{fn.__name__}: {type(e).__name__}: {e}", file=sys.stderr)
                return {"error": f"{type(e).__name__}: {e}"}
            finally:
                torch.cuda.empty_cache()

        t0 = time.perf_counter()
        backward = run_side(bench_backward)
        batched = run_side(bench_batched)
        log(f"backward and batched workloads in {time.perf_counter() - t0:.1f}s")

    out = {
        "metric": METRIC,
        "value": t_solve,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_solve * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage, f64 accumulation" if mixed else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{name}: N={N}, d={d}, "
                         + ("X=G diag(s), s log-spaced 1..1e-6, X,Y float32"
                            if mixed else "X=G diag(s) V^T, s 1..1e-4, 5% rows x100, float64")),
            "sketch": "srht", "r": 6 * d, "m": f"{m[0]}..{m[-1]} x2 (K={len(m)})", "a_i": 2,
            "stage2_steps": s_star, "rel_err": err, "tol": args.tol,
            "resid_grad_GBs": gbs,
            "f64_form": f64,
            "mixed_vs_f64_speedup": (f64["seconds"] / t_solve) if f64 else None,
            "surrogate_stop": surrogate_stop,
            "paper_workloads": paper,
            "backward_workload": backward,
            "batched_workload": batched,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS,
            "traffic": counted_traffic(name),
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": "resid_grad_kernel (fused X^T(Y - X beta), one read of [X|Y])",
            "algorithmic_bytes": bytes_per_sweep,
        },
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
