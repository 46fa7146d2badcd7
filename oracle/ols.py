"""OLS estimator for the oracle (problem statement, Sec. 1).

beta_hat = argmin 1/2 ||Y - X beta||^2 = (X^T X)^{-1} X^T Y, X of full column
rank.  Computed from the Householder QR of [X|Y] (LAPACK dgeqrf through NumPy,
a library primitive): with R_aug = [[R, z], [0, rho]], beta_hat = R^{-1} z and
||Y - X beta_hat|| = |rho|.  Tall inputs are reduced block by block (TSQR:
the QR of the stacked block R factors), so FP32 inputs are promoted one block
at a time.

`ols_refined` adds corrected-seminormal steps (Bjorck): r = Y - X beta and
q = X^T r accumulated in np.longdouble, then R^T R delta = q, beta += delta.
Its result beta_star is the reference for every tolerance.
"""
import numpy as np
from scipy.linalg import solve_triangular

ROW_BLOCK = 1 << 16


def _sign_fix(R):
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return R * s[:, None]


def qr_r(A):
    """Upper-triangular R (nonnegative diagonal) with R^T R = A^T A (Householder)."""
    R = np.linalg.qr(np.asarray(A, np.float64), mode="r")
    return _sign_fix(R)


def tsqr_r(X, Y=None, row_block=ROW_BLOCK):
    """R factor of X (or of [X|Y]) by Householder QR over row blocks."""
    n = X.shape[0]
    R = None
    for i0 in range(0, n, row_block):
        blk = np.asarray(X[i0:i0 + row_block], np.float64)
        if Y is not None:
            blk = np.concatenate([blk, np.asarray(Y[i0:i0 + row_block], np.float64)[:, None]], axis=1)
        Rb = np.linalg.qr(blk, mode="r")
        R = Rb if R is None else np.linalg.qr(np.concatenate([R, Rb], axis=0), mode="r")
    return _sign_fix(R)


def ols_qr(X, Y):
    """(beta_hat, R, rho) from the QR of [X|Y]."""
    d = X.shape[1]
    Raug = tsqr_r(X, Y)
    R = Raug[:d, :d]
    z = Raug[:d, d]
    rho = abs(Raug[d, d]) if Raug.shape[0] > d else 0.0
    beta = solve_triangular(R, z)
    return beta, R, rho


def residual_grad_longdouble(X, Y, beta, row_block=ROW_BLOCK):
    """q = X^T (Y - X beta) with residuals and sums in np.longdouble."""
    d = X.shape[1]
    b = np.asarray(beta, np.longdouble)
    q = np.zeros(d, np.longdouble)
    for i0 in range(0, X.shape[0], row_block):
        Xb = np.asarray(X[i0:i0 + row_block], np.longdouble)
        rb = np.asarray(Y[i0:i0 + row_block], np.longdouble) - Xb @ b
        q += Xb.T @ rb
    return q


def ols_refined(X, Y, steps=3):
    """beta_star: QR solution followed by corrected-seminormal refinement.

    Returns (beta_star, beta_qr, R).
    """
    beta_qr, R, _ = ols_qr(X, Y)
    beta = np.asarray(beta_qr, np.longdouble)
    for _ in range(steps):
        q = residual_grad_longdouble(X, Y, beta)
        qd = np.asarray(q, np.float64)
        delta = solve_triangular(R, solve_triangular(R, qd, trans="T"))
        beta = beta + np.asarray(delta, np.longdouble)
    return np.asarray(beta, np.float64), beta_qr, R


def normal_equation_residual(X, Y, beta):
    """||X^T (Y - X beta)|| in float64 (the fixed-point condition of eq. (99))."""
    Xd = np.asarray(X, np.float64)
    return np.linalg.norm(Xd.T @ (np.asarray(Y, np.float64) - Xd @ beta))
