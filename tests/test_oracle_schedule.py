"""Pins of the oracle's schedule and step-size helpers, its stop estimate, the
prediction error and the IHS baseline (CPU only).

The schedule and step sizes are pinned by the values the experiments state
(Sec. 5: r = 6d, eta = d/r, mu = (1 - eta)^2, m_1 = 8d, m_{i+1} = 2 m_i,
m_K = N/2).  The stop estimate is pinned through an exact Hessian sketch, where
H_hat^{-1} g_t = beta_hat - beta_t holds exactly, so the estimate must equal
||beta_hat - beta_t|| / ||beta_{t+1}|| computed from the OLS solution.  The
prediction error of OLS is pinned by the projection of the noise onto the
column space of X, ||Q^T zeta||^2.  IHS is pinned by its Newton special case
and by its convergence to OLS.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ols as O
from oracle import slse as L
from slse_inputs import make_problem


def test_paper_schedule_stated_values():
    # N = 2^20, d = 2^6: m_1 = 8d = 512 doubling to m_K = N/2 = 2^19, K = log2(N/m_1) = 11
    m = L.paper_schedule(1 << 20, 64)
    assert m == [512 << k for k in range(11)]
    assert len(m) == 11 and m[0] == 8 * 64 and m[-1] == (1 << 20) // 2
    # the mixed workload 2^22 x 512: m = 2^12 .. 2^21, K = 10
    assert L.paper_schedule(1 << 22, 512) == [1 << k for k in range(12, 22)]
    # the ill-conditioned workload 2^20 x 256: m = 2^11 .. 2^19, K = 9
    assert L.paper_schedule(1 << 20, 256) == [1 << k for k in range(11, 20)]


@pytest.mark.parametrize("n,d,first,last", [
    (100000, 70, 1024, 32768),    # 8d = 560 -> 1024; N/2 = 50000 -> 32768
    (100000, 64, 512, 32768),     # 8d a power of 2 is kept
    (1 << 15, 96, 1024, 1 << 14), # 8d = 768 -> 1024
    (70000, 5, 64, 32768),        # 8d = 40 -> 64
    (4096, 1, 8, 2048),
])
def test_paper_schedule_rounding(n, d, first, last):
    m = L.paper_schedule(n, d)
    assert m[0] == first and m[-1] == last
    assert all(b == 2 * a for a, b in zip(m, m[1:]))  # m_{i+1}/m_i = 2
    assert m[0] >= 8 * d and m[0] < 16 * d            # the power of 2 at or above 8d
    assert m[-1] <= n // 2 < 2 * m[-1]                 # the power of 2 at or below N/2


def test_paper_schedule_empty_when_n_too_small():
    assert L.paper_schedule(1000, 100) == []  # 8d = 800 -> 1024 > N/2


@pytest.mark.parametrize("d,r", [(64, 384), (32, 192), (512, 3072), (7, 42)])
def test_default_params_stated_values(d, r):
    mu, eta = L.default_params(d, r)
    # r = 6d gives eta = 1/6 and mu = 25/36 exactly (up to the final rounding)
    eta_x = Fraction(d, r)
    mu_x = (1 - eta_x) ** 2
    assert abs(eta - float(eta_x)) <= 2.0 ** -53 * float(eta_x)
    assert abs(mu - float(mu_x)) <= 4 * 2.0 ** -53 * float(mu_x)
    assert eta_x == Fraction(1, 6) and mu_x == Fraction(25, 36)


def _exact_hessian(s, a0=0, n=256, d=6):
    p = make_problem("plain_small", n=n, d=d)
    # every one of the N' rows kept by the SRHT: H_hat = X^T X up to rounding,
    # and level 1 (all N' rows) has B^T B / N' = X^T X as well
    out = L.slse_frs(p.X, p.Y, 12, "srht", [n], [a0], n, s=s)
    return p, out


@pytest.mark.parametrize("a0", [0, 2])
def test_stop_estimate_is_the_error_for_an_exact_hessian(a0):
    p, (beta, traj, info) = _exact_hessian(s=6, a0=a0)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    sur = info["surrogate"]
    assert len(sur) == a0 + 6 == len(traj) - 1
    for t, v in enumerate(sur):
        want = np.linalg.norm(bstar - traj[t]) / np.linalg.norm(traj[t + 1])
        if want > 1e-10:
            assert abs(v / want - 1) < 1e-9, (t, v, want)
        else:
            assert v < 1e-9


def test_stop_estimate_zero_denominator():
    R = np.eye(3)
    assert L.stop_estimate(R, np.array([3.0, 4.0, 0.0]), np.zeros(3)) == 5.0
    assert L.stop_estimate(2 * R, np.array([4.0, 0.0, 0.0]), np.array([0.0, 2.0, 0.0])) == 0.5


def test_prediction_error_of_ols_is_the_projected_noise():
    g = np.random.default_rng(5)
    n, d = 3000, 9
    X = g.standard_normal((n, d)) * np.logspace(0, -3, d)[None, :]
    beta = g.standard_normal(d)
    zeta = 1e-2 * g.standard_normal(n)
    Y = X @ beta + zeta
    bstar, _, _ = O.ols_refined(X, Y)
    Q, _ = np.linalg.qr(X)
    # X (beta_hat - beta) = P_X zeta, so Delta_LS = ||Q^T zeta||^2 (chi^2_d sigma^2 in law)
    want = float(np.sum((Q.T @ zeta) ** 2))
    got = L.prediction_error(X, bstar, beta, row_block=777)
    assert abs(got / want - 1) < 1e-8
    assert L.prediction_error(X, beta, beta) == 0.0
    # orthonormal columns: ||Q e||^2 = ||e||^2
    e = g.standard_normal(d)
    assert abs(L.prediction_error(Q, e, np.zeros(d)) / float(e @ e) - 1) < 1e-12


def test_ihs_exact_hessian_is_a_newton_step():
    p = make_problem("plain_small", n=512, d=7)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    beta, traj = L.ihs(p.X, p.Y, 40, "srht", 512, steps=1)
    assert L.rel_err(traj[1], bstar) < 1e-12


def test_ihs_refreshes_the_sketch_and_reaches_ols():
    p = make_problem("plain_small", n=8192, d=16)
    bstar, _, _ = O.ols_refined(p.X, p.Y)
    r = 6 * 16
    beta, traj = L.ihs(p.X, p.Y, 300, "srht", r, steps=60)
    assert L.rel_err(beta, bstar) < 1e-14
    errs = np.array([L.rel_err(b, bstar) for b in traj[1:40]])
    rate = np.exp(np.mean(np.diff(np.log(errs))))
    assert rate < 0.7  # a contraction whose size is set by d/r (Sec. 1, IHS)
    # step 0 uses the sketch of key `seed`: the fixed-Hessian iteration with
    # mu = 1, eta = 0 on that key takes the same first step and then departs
    level = 128
    b1, t1, _ = L.slse_frs(p.X, p.Y, 300, "srht", [level], [0], r, s=3, mu=1.0, eta=0.0)
    assert L.rel_err(traj[1], t1[1]) < 1e-14
    assert L.rel_err(traj[2], t1[2]) > 1e-6
