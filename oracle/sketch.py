"""Sketches of the tall data [X|Y] for the oracle.

SRHT (Sec. 3, the SRHT definition and the efficient construction of the
sketched data): S = (N'/m)^{1/2} B H_norm D P over the zero-padded length
N' = 2^ceil(log2 N).  All K nested sketches share one transform
S_0[X|Y] = H D P [X|Y]; sketch i keeps m_i of its rows.  With the unnormalised
H the kept rows carry the factor m_i^{-1/2}, so level i stores the raw rows and
its gradient scale is c_i = 1/m_i.  Sampling reading: exactly m_i rows without
replacement, nested as prefixes of one keyed sample order sigma (the paper's
Bernoulli mask gives a random count but needs nested sets); the Hessian sketch
S_hat (r rows) shares H D P and uses an independent order sigma_hat.

CountSketch (Sec. 1.2, Sec. 5.4): A_K[h(j)] += s(j) [x_j | y_j] with m_K = 2^q
buckets; level i uses the bucket h(j) mod m_i, c_i = 1.  S_hat is an
independent CountSketch with r buckets.

Gaussian (Sec. 1.2): entries N(0, 1/m); the stored rows are G[X|Y] with
G iid N(0,1), levels are prefixes, c_i = 1/m_i.

The returned dict holds
  A       [rows_A, d+1] float64 sketched rows, levels stored by `offset`
  Ahat    [r, d+1]      float64 Hessian-sketch rows
  m, offset, scale      per level; hat_scale (1/r or 1)
"""
import numpy as np

from . import rng
from .fwht import fwht, hadamard_rows


def pad_pow2(n):
    """(p, N') with N' = 2^p the smallest power of 2 >= n (and >= 2)."""
    p = max(1, (int(n) - 1).bit_length())
    return p, 1 << p


def joint(X, Y):
    """[X|Y] as float64 (the sketch acts on both at once, Sec. 3)."""
    return np.concatenate([np.asarray(X, np.float64), np.asarray(Y, np.float64)[:, None]], axis=1)


def _check_levels(m, r, n_limit):
    m = [int(v) for v in m]
    if any(b <= a for a, b in zip(m, m[1:])):
        raise ValueError("sketch sizes must increase")
    if m[-1] > n_limit or r > n_limit:
        raise ValueError("sketch larger than the (padded) row count")
    return m


def srht_transform(X, Y, seed):
    """S_0[X|Y] = H D P [X|Y] (unnormalised H), shape [N', d+1]."""
    W = joint(X, Y)
    n = W.shape[0]
    p, n_pad = pad_pow2(n)
    pi = rng.prp(np.arange(n_pad), seed, rng.STREAM_P, p).astype(np.int64)
    D = rng.rademacher(seed, n_pad).astype(np.float64)
    V = np.zeros((n_pad, W.shape[1]))
    inside = pi < n
    V[inside] = W[pi[inside]]
    V *= D[:, None]
    return fwht(V), p


def srht_orders(seed, p, m_K, r):
    sigma = rng.prp(np.arange(m_K), seed, rng.STREAM_S, p).astype(np.int64)
    sigma_hat = rng.prp(np.arange(r), seed, rng.STREAM_SHAT, p).astype(np.int64)
    return sigma, sigma_hat


def srht(X, Y, seed, m, r):
    n = len(Y)
    p, n_pad = pad_pow2(n)
    m = _check_levels(m, r, n_pad)
    Z, p = srht_transform(X, Y, seed)
    sigma, sigma_hat = srht_orders(seed, p, m[-1], r)
    return dict(A=Z[sigma], Ahat=Z[sigma_hat], m=m, offset=[0] * len(m),
                scale=[1.0 / v for v in m], hat_scale=1.0 / r, n_pad=n_pad)


def srht_rows(X, Y, seed, rows):
    """Rows `rows` of S_0[X|Y] one by one from the popcount formula (no FWHT).

    Used to check sampled output rows of a large transform.
    """
    W = joint(X, Y)
    n = W.shape[0]
    p, n_pad = pad_pow2(n)
    pi = rng.prp(np.arange(n_pad), seed, rng.STREAM_P, p).astype(np.int64)
    D = rng.rademacher(seed, n_pad).astype(np.float64)
    out = np.zeros((len(rows), W.shape[1]))
    chunk = 1 << 16
    for k0 in range(0, n_pad, chunk):
        k = np.arange(k0, min(n_pad, k0 + chunk))
        src = pi[k]
        ok = src < n
        V = np.zeros((len(k), W.shape[1]))
        V[ok] = W[src[ok]]
        V *= D[k][:, None]
        Hs = hadamard_rows(rows, n_pad, k)
        out += Hs @ V
    return out


def countsketch(X, Y, seed, m, r):
    W = joint(X, Y)
    n = W.shape[0]
    m = _check_levels(m, r, max(n, m[-1]))
    for v in m:
        if v & (v - 1):
            raise ValueError("CountSketch levels must be powers of 2")
    h, s = rng.countsketch_hash(seed, n, m[-1])
    SW = W * s[:, None].astype(np.float64)
    blocks, offset, off = [], [], 0
    for v in m:
        Ai = np.zeros((v, W.shape[1]))
        np.add.at(Ai, h & (v - 1), SW)
        blocks.append(Ai)
        offset.append(off)
        off += v
    hh, ss = rng.countsketch_hash_hat(seed, n, r)
    Ahat = np.zeros((r, W.shape[1]))
    np.add.at(Ahat, hh, W * ss[:, None].astype(np.float64))
    return dict(A=np.concatenate(blocks, axis=0), Ahat=Ahat, m=m, offset=offset,
                scale=[1.0] * len(m), hat_scale=1.0)


def round_to(a, kind):
    """Round float64 values to float32 or bfloat16 (nearest-even), as float64."""
    a = np.asarray(a, np.float64)
    if kind == "f64":
        return a
    f = a.astype(np.float32)
    if kind == "f32":
        return f.astype(np.float64)
    if kind == "bf16":
        u = f.view(np.uint32).astype(np.uint64)
        lsb = (u >> np.uint64(16)) & np.uint64(1)
        u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(kind)


def gaussian_apply(W, seed, stream, m, g_round="f64", col_block=4096):
    """G[0:m] @ W with G_kj iid N(0,1) from the counter stream (entries rounded to g_round)."""
    n = W.shape[0]
    out = np.zeros((m, W.shape[1]))
    k = np.arange(m)
    for j0 in range(0, n, col_block):
        j = np.arange(j0, min(n, j0 + col_block))
        G = round_to(rng.gaussian_block(seed, stream, k, j), g_round)
        out += G @ W[j]
    return out


def gaussian(X, Y, seed, m, r, g_round="f64"):
    W = joint(X, Y)
    m = _check_levels(m, r, 1 << 62)
    A = gaussian_apply(W, seed, rng.STREAM_G, m[-1], g_round)
    Ahat = gaussian_apply(W, seed, rng.STREAM_GHAT, r, g_round)
    return dict(A=A, Ahat=Ahat, m=m, offset=[0] * len(m),
                scale=[1.0 / v for v in m], hat_scale=1.0 / r)


def sketch(kind, X, Y, seed, m, r, **kw):
    if kind == "srht":
        return srht(X, Y, seed, m, r)
    if kind == "countsketch":
        return countsketch(X, Y, seed, m, r)
    if kind == "gaussian":
        return gaussian(X, Y, seed, m, r, **kw)
    raise ValueError(kind)
