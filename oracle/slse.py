"""The SLSE-FRS iteration for the oracle (Alg. 2, eqs. (98) and (99)).

Stage 1 runs a_i M-IHS steps on each sketched subproblem i = 1..K,

    beta_{t+1} = beta_t - mu H_hat^{-1} grad f(beta_t; S_i X, S_i Y) + eta (beta_t - beta_{t-1}),

and stage 2 runs s full-data steps of the same form (eq. (99)), with
grad f(beta; X, Y) = X^T (X beta - Y) (Sec. 1) and the fixed Hessian sketch
H_hat = (S_hat X)^T S_hat X (Sec. 3) applied through its QR factor R:
H_hat^{-1} v = R^{-1} R^{-T} v (implementation details appendix).

Readings where the paper is silent:
  * beta_0 = 0 and beta_{-1} = beta_0;
  * momentum carries across subproblems and into stage 2 (Alg. 2 keeps one
    global t); `momentum_reset=True` restarts it at each subproblem instead,
    as the proofs do;
  * the stage-2 loop "for t = T_dagger to T" is read as exactly s steps;
  * defaults mu = (1 - eta)^2, eta = d / r (Sec. 5 parameter choice).
The gradient is formed in residual form g = c X^T (Y - X beta) = -c grad f and
added with +mu.
"""
import math

import numpy as np
from scipy.linalg import solve_triangular

from .ols import qr_r
from .sketch import sketch as make_sketch

ROW_BLOCK = 1 << 16


def default_params(d, r):
    """(mu, eta) = ((1 - d/r)^2, d/r), the step sizes of the experiments (Sec. 5,
    following the M-IHS choice)."""
    eta = d / r
    return (1.0 - eta) ** 2, eta


def precond_factor(Ahat, d, hat_scale):
    """R with R^T R = hat_scale * Ahat[:, :d]^T Ahat[:, :d] (Householder QR)."""
    return qr_r(np.sqrt(hat_scale) * np.asarray(Ahat[:, :d], np.float64))


def apply_precond(R, v):
    """H_hat^{-1} v = R^{-1} (R^{-T} v)."""
    return solve_triangular(R, solve_triangular(R, v, trans="T"))


def sketched_grad(Ai, d, c, beta):
    """c * B^T (b - B beta) for the sketched rows Ai = [B | b]."""
    B = Ai[:, :d]
    return c * (B.T @ (Ai[:, d] - B @ beta))


def full_grad(X, Y, beta, row_block=ROW_BLOCK):
    """X^T (Y - X beta) in float64, streamed over row blocks."""
    d = X.shape[1]
    g = np.zeros(d)
    for i0 in range(0, X.shape[0], row_block):
        Xb = np.asarray(X[i0:i0 + row_block], np.float64)
        Yb = np.asarray(Y[i0:i0 + row_block], np.float64)
        g += Xb.T @ (Yb - Xb @ beta)
    return g


def mihs_step(beta, beta_prev, g, R, mu, eta):
    return beta + mu * apply_precond(R, g) + eta * (beta - beta_prev)


def stop_estimate(R, g, beta_next):
    """Estimate of the relative error of beta_t that a step can report for free:
    ||H_hat^{-1} g_t|| / ||beta_{t+1}||.  At the fixed point of eq. (99) the
    full-data gradient is X^T X (beta_hat - beta_t), so with H_hat ~ X^T X the
    numerator approximates ||beta_hat - beta_t||.  A zero denominator leaves
    the bare numerator."""
    num = float(np.linalg.norm(apply_precond(R, g)))
    den = float(np.linalg.norm(beta_next))
    return num / den if den > 0.0 else num


def prediction_error(X, beta, beta_ref, row_block=ROW_BLOCK):
    """Delta = ||X (beta - beta_ref)||^2, the error measure of the experiments
    (Sec. 5, with beta_ref the true coefficient vector), streamed over row
    blocks in float64."""
    e = np.asarray(beta, np.float64) - np.asarray(beta_ref, np.float64)
    tot = 0.0
    for i0 in range(0, X.shape[0], row_block):
        v = np.asarray(X[i0:i0 + row_block], np.float64) @ e
        tot += float(v @ v)
    return tot


def slse_frs(X, Y, seed, kind, m, a, r, s, mu=None, eta=None, beta0=None,
             momentum_reset=False, sk=None, start=0, stop=None, beta_prev0=None, **sketch_kw):
    """Run Alg. 2 and return (beta_T, trajectory, info).

    trajectory[t] is beta_t for t = 0..T (T = sum(a) + s).  info["surrogate"][t]
    is stop_estimate of step t (the step from beta_t to beta_{t+1}, with the
    scaled sketched gradient in stage 1).  `sk` may pass a precomputed oracle
    sketch (same seed and sizes) to avoid recomputing it.

    Checkpoint and resume: the steps are numbered t = 0..T-1 over the whole
    algorithm (stage 1 level by level, then stage 2), and the sketch is a
    function of the seed, so the iteration's whole state after step t - 1 is
    (beta_t, beta_{t-1}).  With start > 0 the call runs steps start..stop-1
    from beta_start = beta0 and beta_{start-1} = beta_prev0 (beta0 when None);
    trajectory and surrogate entries before `start` are None.  A momentum
    reset at the start of a subproblem (or of stage 2) happens when the first
    step of that subproblem is run.  info["state"] = (beta_{t-1}, beta_t) at
    the last iterate t computed, the checkpoint to resume from.
    """
    d = X.shape[1]
    if mu is None or eta is None:
        mu0, eta0 = default_params(d, r)
        mu = mu0 if mu is None else mu
        eta = eta0 if eta is None else eta
    if sk is None:
        sk = make_sketch(kind, X, Y, seed, m, r, **sketch_kw)
    R = precond_factor(sk["Ahat"], d, sk["hat_scale"])
    T = sum(a[: len(sk["m"])]) + s
    stop = T if stop is None else stop
    assert 0 <= start <= stop <= T
    beta = np.zeros(d) if beta0 is None else np.asarray(beta0, np.float64).copy()
    beta_prev = beta.copy() if beta_prev0 is None else np.asarray(beta_prev0, np.float64).copy()
    traj = [None] * start + [beta.copy()]
    sur = [None] * start
    # the step sequence of Alg. 2: (subproblem or None for stage 2, its first step?)
    steps = []
    for i, ai in enumerate(a[: len(sk["m"])]):
        steps += [(i, j == 0) for j in range(ai)]
    steps += [(None, j == 0) for j in range(s)]
    # a reset at a subproblem with no steps is repeated by the next one's: no effect
    for t in range(start, stop):
        i, first = steps[t]
        if momentum_reset and first:
            beta_prev = beta.copy()
        if i is not None:
            Ai = sk["A"][sk["offset"][i]: sk["offset"][i] + sk["m"][i]]
            g = sketched_grad(Ai, d, sk["scale"][i], beta)
        else:
            g = full_grad(X, Y, beta)
        beta, beta_prev = mihs_step(beta, beta_prev, g, R, mu, eta), beta
        sur.append(stop_estimate(R, g, beta))
        traj.append(beta.copy())
    return beta, traj, dict(R=R, sketch=sk, mu=mu, eta=eta, surrogate=sur,
                            state=(beta_prev.copy(), beta.copy()))


def ihs(X, Y, seed, kind, r, steps, beta0=None, **sketch_kw):
    """Iterative Hessian sketch with the Hessian sketch drawn anew at every
    step (the IHS update of Sec. 1, the baseline that SLSE-FRS improves on):

        beta_{t+1} = beta_t + H_t^{-1} X^T (Y - X beta_t),
        H_t = (S_t X)^T S_t X,

    i.e. eq. (99) with mu = 1, eta = 0 and a fresh S_t of r rows per step.
    Step t draws S_t with sketch key seed + t and uses the Hessian-sketch rows
    (Ahat) of that key, so every step's sketch is independent of the others.
    The sketch call also forms one nested level, which IHS does not use; its
    size is the power of 2 >= r (a valid level for every sketch family).
    Returns (beta_T, trajectory)."""
    d = X.shape[1]
    level = 1 << max(0, (int(r) - 1).bit_length())
    beta = np.zeros(d) if beta0 is None else np.asarray(beta0, np.float64).copy()
    traj = [beta.copy()]
    for t in range(steps):
        sk = make_sketch(kind, X, Y, seed + t, [level], r, **sketch_kw)
        R = precond_factor(sk["Ahat"], d, sk["hat_scale"])
        g = full_grad(X, Y, beta)
        beta = beta + apply_precond(R, g)
        traj.append(beta.copy())
    return beta, traj


def iteration_lower_bounds(m, d, omega):
    """Real lower bounds of the stage-1 counts a_2..a_K (Thm lowerBoundai, Sec. 4):
    a_i >= log_3[((1 + omega) r(i-1, i) + 1) / omega] with
    r(i-1, i) = sqrt((m_i - d) / (m_{i-1} - d)).  Entry 0 (a_1) is None: its
    bound (Thm a1, Appendix) needs the unknown errors of the first subproblem."""
    out = [None]
    for i in range(1, len(m)):
        ratio = math.sqrt((m[i] - d) / (m[i - 1] - d))
        out.append(math.log(((1.0 + omega) * ratio + 1.0) / omega) / math.log(3.0))
    return out


def paper_schedule(n, d, m1_factor=8):
    """m_1 = 8d, m_{i+1} = 2 m_i, m_K = the largest power of 2 <= N/2 (Sec. 5, Sec. 3).

    When 8d is not a power of 2 the schedule starts at the power of 2 above it.
    """
    m1 = 1 << max(0, (m1_factor * d - 1).bit_length())
    mk = 1 << ((n // 2).bit_length() - 1)
    m = []
    v = m1
    while v <= mk:
        m.append(v)
        v *= 2
    return m


def rel_err(beta, ref):
    return float(np.linalg.norm(np.asarray(beta) - ref) / np.linalg.norm(ref))
