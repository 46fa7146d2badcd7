"""Adjoint of the OLS map for the oracle.

For L = w^T beta_hat with beta_hat = (X^T X)^{-1} X^T Y (problem statement,
Sec. 1), differentiating the normal equations gives, with
lambda = (X^T X)^{-1} w and r = Y - X beta_hat,

    dL/dY = X lambda,        dL/dX = r lambda^T - (X lambda) beta_hat^T.

Here lambda = R^{-1} R^{-T} w with R from the Householder QR of X.
`fd_gradient` is the independent check: central differences of
w^T beta_hat over every entry of a small problem, with QR solves.
"""
import numpy as np
from scipy.linalg import solve_triangular

from .ols import ols_refined


def adjoint(X, Y, w, beta_star=None, R=None):
    """(dX, dY, lambda, beta_hat) in float64."""
    Xd = np.asarray(X, np.float64)
    Yd = np.asarray(Y, np.float64)
    if beta_star is None or R is None:
        beta_star, _, R = ols_refined(Xd, Yd)
    lam = solve_triangular(R, solve_triangular(R, np.asarray(w, np.float64), trans="T"))
    u = Xd @ lam
    r = Yd - Xd @ beta_star
    dX = np.outer(r, lam) - np.outer(u, beta_star)
    return dX, u, lam, beta_star


def _ols_solve(X, Y):
    Q, R = np.linalg.qr(X)
    return solve_triangular(R, Q.T @ Y)


def fd_gradient(X, Y, w, h=None):
    """Central-difference dL/dX and dL/dY of L = w^T beta_hat (small problems)."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    if h is None:
        h = 6e-6
    n, d = X.shape
    dX = np.zeros_like(X)
    dY = np.zeros_like(Y)
    for i in range(n):
        for j in range(d):
            hp = h * max(1.0, abs(X[i, j]))
            Xp = X.copy()
            Xp[i, j] += hp
            Xm = X.copy()
            Xm[i, j] -= hp
            dX[i, j] = (w @ _ols_solve(Xp, Y) - w @ _ols_solve(Xm, Y)) / (2 * hp)
        hp = h * max(1.0, abs(Y[i]))
        Yp = Y.copy()
        Yp[i] += hp
        Ym = Y.copy()
        Ym[i] -= hp
        dY[i] = (w @ _ols_solve(X, Yp) - w @ _ols_solve(X, Ym)) / (2 * hp)
    return dX, dY
