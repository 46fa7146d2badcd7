"""Pins of the oracle's OLS, SLSE-FRS iteration and adjoint (CPU only).

OLS is pinned by exact rational arithmetic on tiny integer problems, the
normal equations and recovery of a planted beta.  The iteration is pinned by
special cases with closed forms: with an exact Hessian sketch (every SRHT row
kept, so H_hat = X^T X) one step with mu = 1, eta = 0 is a Newton step and
lands on beta_hat; with eta != 0 the error obeys e_{t+1} = (1-mu) e_t +
eta (e_t - e_{t-1}); stage 1 run long converges to the sketch-and-solve
estimator of the last subproblem; stage 2 converges to beta_hat at about the
M-IHS rate sqrt(d/r).  The adjoint is pinned by its two invariants and by
central finite differences.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import adjoint as ADJ
from oracle import ols as O
from oracle import sketch as S
from oracle import slse as L
from slse_inputs import make_problem, paper_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _solve_fraction(A, b):
    """Gaussian elimination over the rationals."""
    n = len(b)
    M = [[Fraction(int(v)) for v in row] + [Fraction(int(bi))] for row, bi in zip(A, b)]
    for c in range(n):
        piv = next(i for i in range(c, n) if M[i][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for i in range(n):
            if i != c and M[i][c] != 0:
                f = M[i][c] / M[c][c]
                M[i] = [a - f * bb for a, bb in zip(M[i], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


@pytest.mark.parametrize("seed", range(6))
def test_ols_exact_rational(seed):
    g = np.random.default_rng(seed)
    n, d = 8, 3
    X = g.integers(-5, 6, size=(n, d))
    Y = g.integers(-9, 10, size=n)
    exact = _solve_fraction(X.T @ X, X.T @ Y)
    beta, _, _ = O.ols_qr(X.astype(float), Y.astype(float))
    bstar, _, _ = O.ols_refined(X.astype(float), Y.astype(float))
    ex = np.array([float(v) for v in exact])
    np.testing.assert_allclose(beta, ex, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(bstar, ex, rtol=1e-15, atol=1e-15)


def test_ols_normal_equations_and_tsqr_blocks():
    p = make_problem("plain_small", n=5000, d=12)
    beta, R, rho = O.ols_qr(p.X, p.Y)
    u = 2.0 ** -53
    nx = np.linalg.norm(p.X, 2)
    bound = 50 * u * nx * (nx * np.linalg.norm(beta) + np.linalg.norm(p.Y))
    assert O.normal_equation_residual(p.X, p.Y, beta) < bound
    np.testing.assert_allclose(rho, np.linalg.norm(p.Y - p.X @ beta), rtol=1e-10)
    R2 = O.tsqr_r(p.X, row_block=777)
    np.testing.assert_allclose(R2, R, rtol=1e-10, atol=1e-10)


def test_ols_planted_beta_recovered():
    g = np.random.default_rng(3)
    X = g.standard_normal((2000, 10)) * np.logspace(0, -4, 10)[None, :]
    beta = g.standard_normal(10)
    Y = X @ beta
    bstar, bqr, _ = O.ols_refined(X, Y)
    kappa = np.linalg.cond(X)
    assert L.rel_err(bqr, beta) < 100 * kappa * 2.0 ** -53
    assert L.rel_err(bstar, beta) < 1e-14


def test_ols_agrees_with_lapack_lstsq():
    p = make_problem("illcond", n=20000, d=24)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    ref = np.linalg.lstsq(p.X, p.Y, rcond=None)[0]
    assert L.rel_err(ref, bstar) < 1e-10


def _exact_hessian_run(kind_eta, mu, s=6):
    p = make_problem("plain_small", n=256, d=6)
    # every one of the N' rows kept: S_hat^T S_hat = I, so H_hat = X^T X
    return p, L.slse_frs(p.X, p.Y, 12, "srht", [256], [0], 256, s=s, mu=mu, eta=kind_eta)


def test_exact_hessian_newton_step_lands_on_ols():
    p, (beta, traj, _) = _exact_hessian_run(0.0, 1.0, s=1)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    assert L.rel_err(traj[1], bstar) < 1e-12


@pytest.mark.parametrize("mu,eta", [(0.5, 0.0), (1.0, 0.3), (0.7, 0.2)])
def test_exact_hessian_error_recursion(mu, eta):
    p, (beta, traj, _) = _exact_hessian_run(eta, mu, s=8)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    e = [traj[0] - bstar, traj[0] - bstar]  # e_{-1} = e_0 (beta_{-1} = beta_0)
    for t in range(8):
        e.append((1 - mu) * e[-1] + eta * (e[-1] - e[-2]))
    for t in range(9):
        np.testing.assert_allclose(traj[t] - bstar, e[t + 1], atol=1e-10)


@pytest.mark.parametrize("kind", ["srht", "countsketch", "gaussian"])
def test_stage1_limit_is_sketch_and_solve(kind):
    p = make_problem("plain_small", n=2048, d=8)
    m, r = [64, 128], 48
    sk = S.sketch(kind, p.X, p.Y, 21, m, r)
    beta, traj, info = L.slse_frs(p.X, p.Y, 21, kind, m, [0, 120], r, s=0, sk=sk)
    A = sk["A"][sk["offset"][1]: sk["offset"][1] + 128]
    tilde = np.linalg.lstsq(A[:, :8], A[:, 8], rcond=None)[0]
    assert L.rel_err(beta, tilde) < 1e-10
    assert L.rel_err(beta, O.ols_refined(p.X, p.Y)[0]) > 1e-6  # it is not OLS


@pytest.mark.parametrize("kind", ["srht", "countsketch"])
def test_stage2_fixed_point_and_rate(kind):
    p = make_problem("plain_small")
    d, r = 32, 192
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    m = [64, 128, 256, 512, 1024]
    beta, traj, _ = L.slse_frs(p.X, p.Y, 1001, kind, m, [2] * 5, r, s=45)
    assert L.rel_err(beta, bstar) < 1e-14
    errs = np.array([L.rel_err(b, bstar) for b in traj[10:35]])
    rate = np.exp(np.mean(np.diff(np.log(errs))))
    assert rate < 0.6  # M-IHS rate ~ sqrt(d/r) = 0.41 (Sec. 1, Ozaslan et al.)


def test_momentum_reset_changes_only_the_path():
    p = make_problem("plain_small", n=4096, d=16)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    m = [128, 256, 512]
    b1, t1, _ = L.slse_frs(p.X, p.Y, 5, "srht", m, [2] * 3, 96, s=40)
    b2, t2, _ = L.slse_frs(p.X, p.Y, 5, "srht", m, [2] * 3, 96, s=40, momentum_reset=True)
    assert not np.allclose(t1[3], t2[3])
    assert L.rel_err(b1, bstar) < 1e-13 and L.rel_err(b2, bstar) < 1e-13


@pytest.mark.parametrize("reset", [False, True])
def test_checkpoint_resume_is_bit_identical(reset):
    # the state after step t - 1 is (beta_t, beta_{t-1}) (the sketch is a
    # function of the seed): a run stopped at k and resumed from its state
    # retraces the uninterrupted run exactly, mid-subproblem, at a subproblem
    # boundary, at the start of stage 2, inside stage 2 and at the end
    p = make_problem("plain_small", n=2048, d=12)
    m, a, r, s = [128, 256, 512], [2, 3, 2], 72, 9
    sk = S.sketch("srht", p.X, p.Y, 33, m, r)
    b_full, t_full, _ = L.slse_frs(p.X, p.Y, 33, "srht", m, a, r, s, sk=sk, momentum_reset=reset)
    T = sum(a) + s
    for k in [0, 1, 2, 3, 5, 7, 8, 12, T - 1, T]:
        _, t_part, info = L.slse_frs(p.X, p.Y, 33, "srht", m, a, r, s, sk=sk, stop=k,
                                     momentum_reset=reset)
        prev, cur = info["state"]
        assert np.array_equal(cur, t_full[k])
        if k > 0:
            assert np.array_equal(prev, t_full[k - 1])
        b_res, t_res, _ = L.slse_frs(p.X, p.Y, 33, "srht", m, a, r, s, sk=sk, start=k, beta0=cur,
                                     beta_prev0=prev, momentum_reset=reset)
        assert np.array_equal(b_res, b_full), k
        for t in range(k, T + 1):
            assert np.array_equal(t_res[t], t_full[t]), (k, t)
    # a resume that forgets beta_{t-1} loses the momentum term: another path
    _, t_bad, _ = L.slse_frs(p.X, p.Y, 33, "srht", m, a, r, s, sk=sk, start=3, beta0=t_full[3])
    assert not np.allclose(t_bad[4], t_full[4])


def test_paper_ls_error_level():
    """Delta_T reaches the LS error sigma^2 d (Sec. 5.2 and its Fig. 2 left)."""
    with open(os.path.join(GOLDEN, "paper_ls_error.json")) as f:
        gold = json.load(f)
    p = paper_problem(gold["N"], gold["d"], gold["kappa"], sigma2=gold["sigma2"])
    d, r = gold["d"], 6 * gold["d"]
    m = L.paper_schedule(gold["N"], d)
    beta, traj, _ = L.slse_frs(p.X, p.Y, 7, "srht", m, [2] * len(m), r, s=gold["stage2_steps"])
    delta_T = float(np.sum((p.X @ (beta - p.beta_true)) ** 2))
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    delta_ls = float(np.sum((p.X @ (bstar - p.beta_true)) ** 2))
    # the printed level sigma^2 d = 6.4e-7 (chi^2_d spread: +-50% is > 3 sd)
    assert abs(delta_ls / gold["ls_error"] - 1) < 0.5
    assert abs(delta_T / delta_ls - 1) < 1e-3


def test_adjoint_invariants():
    p = make_problem("backward", n=3000, d=10)
    w = np.random.default_rng(0).standard_normal(10)
    dX, dY, lam, bstar = ADJ.adjoint(p.X, p.Y, w)
    X = p.X.astype(np.float64)
    np.testing.assert_allclose(X.T @ dY, w, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(X.T @ dX, -np.outer(w, bstar), rtol=1e-8, atol=1e-9)


def test_adjoint_matches_finite_differences():
    g = np.random.default_rng(4)
    X = g.standard_normal((40, 4))
    Y = X @ g.standard_normal(4) + 0.1 * g.standard_normal(40)
    w = g.standard_normal(4)
    dX, dY, _, _ = ADJ.adjoint(X, Y, w)
    fX, fY = ADJ.fd_gradient(X, Y, w)
    np.testing.assert_allclose(dX, fX, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(dY, fY, rtol=1e-6, atol=1e-8)


def test_iteration_lower_bounds_and_binding_schedule():
    # Thm lowerBoundai: a_i >= log_3[((1 + w) r + 1) / w], r = sqrt((m_i - d)/(m_{i-1} - d))
    import math

    from oracle import slse as OS
    from paper_2509_06856_amd.slse import auto_a

    d = 64
    m = [512 * 2 ** k for k in range(8)]
    for w in (1 / 16, 1 / 8, 1 / 4, 1 / 2, 1.0):
        lb = OS.iteration_lower_bounds(m, d, w)
        assert lb[0] is None
        # the integer schedule is the ceiling of the real bound
        a = auto_a(m, d, w, a1=7)
        assert a[0] == 7 and a[1:] == [math.ceil(x - 1e-12) for x in lb[1:]]
    # closed form: a doubling schedule has r -> sqrt(2) as m grows, so at w = 1/2
    # the bound tends to log_3(6.24...) < 2 (the paper's a_i = 2 recommendation)
    big = [2 ** 20, 2 ** 21]
    lb = OS.iteration_lower_bounds(big, d, 0.5)[1]
    assert abs(lb - math.log((1.5 * math.sqrt((2 ** 21 - d) / (2 ** 20 - d)) + 1) / 0.5, 3)) < 1e-12
    assert 1.6 < lb < 1.7
    # the bound falls as the tolerance w grows (Fig. on the determination of a_i)
    vals = [OS.iteration_lower_bounds(m, d, w)[2] for w in (1 / 16, 1 / 8, 1 / 4, 1 / 2, 1.0)]
    assert all(x > y for x, y in zip(vals, vals[1:]))
    # equal consecutive sizes (r = 1) give log_3((2 + w)/w): w = 1 -> exactly 1
    assert abs(OS.iteration_lower_bounds([1000, 1000], 10, 1.0)[1] - 1.0) < 1e-12
