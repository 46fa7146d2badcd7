"""Counter-based randomness of the sketches, written for the oracle.

The paper draws the SRHT's Rademacher diagonal D, the uniform permutation P and
the row sampling B at random (Sec. 3, the SRHT definition), the CountSketch's
one +-1 per column (Sec. 1.2 and Sec. 5.4) and the Gaussian sketch's iid
entries (Sec. 1.2).  It does not say how.  Here every one of them is drawn
from Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), keyed by (seed, stream), so that any single entry can
be recomputed from its index alone.

Stream map (key word 1):
  1 D signs     2 permutation P     3 sample order sigma (sketches S_i)
  4 sample order sigma_hat (Hessian sketch S_hat)
  5 CountSketch of S_K   6 CountSketch of S_hat
  7 Gaussian S   8 Gaussian S_hat

Everything here is vectorised NumPy on uint64 arrays; 64x64->128-bit products
are built from 32-bit halves.
"""
import numpy as np

U64 = np.uint64
M32 = U64(0xFFFFFFFF)

# Philox4x64 round multipliers and Weyl key increments (SC'11, Table/Sec. 5).
PHILOX_M0 = U64(0xD2E7470EE14C6C93)
PHILOX_M1 = U64(0xCA5A826395121157)
PHILOX_W0 = U64(0x9E3779B97F4A7C15)
PHILOX_W1 = U64(0xBB67AE8584CAA73B)

STREAM_D = 1
STREAM_P = 2
STREAM_S = 3
STREAM_SHAT = 4
STREAM_CS = 5
STREAM_CSHAT = 6
STREAM_G = 7
STREAM_GHAT = 8

FEISTEL_ROUNDS = 4


def _u64(a):
    return np.asarray(a, dtype=np.uint64)


def mulhilo64(a, b):
    """(hi, lo) words of the 128-bit product a*b of uint64 arrays."""
    a = _u64(a)
    b = _u64(b)
    a_lo = a & M32
    a_hi = a >> U64(32)
    b_lo = b & M32
    b_hi = b >> U64(32)
    p_ll = a_lo * b_lo
    p_lh = a_lo * b_hi
    p_hl = a_hi * b_lo
    p_hh = a_hi * b_hi
    mid = (p_ll >> U64(32)) + (p_lh & M32) + (p_hl & M32)
    hi = p_hh + (p_lh >> U64(32)) + (p_hl >> U64(32)) + (mid >> U64(32))
    lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=10):
    """Philox4x64-R block function on broadcastable uint64 arrays.

    One round maps (x0, x1, x2, x3) to (hi(M1*x2)^x1^k0, lo(M1*x2),
    hi(M0*x0)^x3^k1, lo(M0*x0)); the key is bumped by the Weyl constants
    between rounds.  Returns the four output words.
    """
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (_u64(c) for c in (c0, c1, c2, c3))
        k0 = _u64(k0)
        k1 = _u64(k1)
        x0, x1, x2, x3, k0, k1 = np.broadcast_arrays(x0, x1, x2, x3, k0, k1)
        x0, x1, x2, x3 = (v.copy() for v in (x0, x1, x2, x3))
        k0 = k0.copy()
        k1 = k1.copy()
        for r in range(rounds):
            if r > 0:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = mulhilo64(PHILOX_M0, x0)
            hi1, lo1 = mulhilo64(PHILOX_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        return x0, x1, x2, x3


def stream_words(seed, stream, c0, c1=0):
    """Philox4x64-10 words at counter (c0, c1, 0, 0) under key (seed, stream)."""
    return philox4x64(c0, c1, 0, 0, U64(seed), U64(stream))


# ----------------------------------------------------------------------------
# D: Rademacher diagonal (SRHT definition, Sec. 3).  256 signs per block:
# row j uses bit (j & 63) of word ((j >> 6) & 3) of block j >> 8.
# ----------------------------------------------------------------------------
def rademacher(seed, n):
    """D_jj in {+1, -1} for j < n, as int8."""
    j = np.arange(n, dtype=np.uint64)
    blocks = np.arange((n + 255) // 256, dtype=np.uint64)
    w = np.stack(stream_words(seed, STREAM_D, blocks), axis=1)  # [blocks, 4]
    word = w[(j >> U64(8)).astype(np.int64), ((j >> U64(6)) & U64(3)).astype(np.int64)]
    bit = (word >> (j & U64(63))) & U64(1)
    return (1 - 2 * bit.astype(np.int64)).astype(np.int8)


# ----------------------------------------------------------------------------
# Keyed permutation of [0, 2^p): a balanced Feistel network on 2h bits,
# h = ceil(p/2), with round function F_i(x) = low h bits of word 0 of
# Philox(ctr=(x, i), key=(seed, stream)); when 2h > p the permutation is
# restricted to [0, 2^p) by cycle walking (Black and Rogaway, CT-RSA 2002).
# The paper asks for a uniform permutation and uniform sampling without
# replacement; this is a pseudo-random stand-in with the same role.
# ----------------------------------------------------------------------------
def _feistel_half_bits(p):
    return (p + 1) // 2


def _feistel_encrypt(x, seed, stream, h):
    mask = U64((1 << h) - 1)
    left = x >> U64(h)
    right = x & mask
    for i in range(FEISTEL_ROUNDS):
        f = stream_words(seed, stream, right, i)[0] & mask
        left, right = right, left ^ f
    return (left << U64(h)) | right


def _feistel_decrypt(y, seed, stream, h):
    mask = U64((1 << h) - 1)
    left = y >> U64(h)
    right = y & mask
    for i in reversed(range(FEISTEL_ROUNDS)):
        f = stream_words(seed, stream, left, i)[0] & mask
        left, right = right ^ f, left
    return (left << U64(h)) | right


def prp(x, seed, stream, p):
    """pi(x) for a keyed permutation pi of [0, 2^p); x is an index array."""
    x = _u64(x).copy()
    h = _feistel_half_bits(p)
    lim = U64(1 << p)
    y = _feistel_encrypt(x, seed, stream, h)
    out_of_range = y >= lim
    while np.any(out_of_range):
        y[out_of_range] = _feistel_encrypt(y[out_of_range], seed, stream, h)
        out_of_range = y >= lim
    return y


def prp_inverse(y, seed, stream, p):
    """pi^{-1}(y) for the permutation of prp()."""
    y = _u64(y).copy()
    h = _feistel_half_bits(p)
    lim = U64(1 << p)
    x = _feistel_decrypt(y, seed, stream, h)
    out_of_range = x >= lim
    while np.any(out_of_range):
        x[out_of_range] = _feistel_decrypt(x[out_of_range], seed, stream, h)
        out_of_range = x >= lim
    return x


# ----------------------------------------------------------------------------
# CountSketch (Sec. 1.2, Sec. 5.4): column j of S has one entry s(j) in row
# h(j).  For the nested sketches S_K has m_K = 2^q rows and h(j) is the low q
# bits of word 0; level i keeps the low log2(m_i) bits.  The Hessian sketch
# S_hat has r rows (any r) and uses the multiply-high reduction
# ((w0 >> 32) * r) >> 32 of Lemire ("Fast random integer generation in an
# interval", TOMACS 2019).
# ----------------------------------------------------------------------------
def countsketch_hash(seed, n, m_pow2):
    j = np.arange(n, dtype=np.uint64)
    w0, w1, _, _ = stream_words(seed, STREAM_CS, j)
    h = (w0 & U64(m_pow2 - 1)).astype(np.int64)
    s = (1 - 2 * (w1 & U64(1)).astype(np.int64)).astype(np.int8)
    return h, s


def countsketch_hash_hat(seed, n, r):
    j = np.arange(n, dtype=np.uint64)
    w0, w1, _, _ = stream_words(seed, STREAM_CSHAT, j)
    with np.errstate(over="ignore"):
        h = (((w0 >> U64(32)) * U64(r)) >> U64(32)).astype(np.int64)
    s = (1 - 2 * (w1 & U64(1)).astype(np.int64)).astype(np.int8)
    return h, s


# ----------------------------------------------------------------------------
# Gaussian sketch (Sec. 1.2): G_kj iid N(0, 1).  Entry (k, j) comes from block
# Philox(ctr=(j, k >> 3), key=(seed, stream)); its 4 words give 4 Box-Muller
# pairs, word q = (k & 7) >> 1 holding u1 in its low and u2 in its high half,
# u = (w32 + 1/2) / 2^32; even k takes the cosine, odd k the sine.
# ----------------------------------------------------------------------------
def gaussian_block(seed, stream, k_rows, j_cols):
    """G[k, j] in float64 for row indices k (array) and column indices j (array)."""
    k = np.asarray(k_rows, dtype=np.int64)
    j = _u64(j_cols)[None, :]
    kb, kb_idx = np.unique(k >> 3, return_inverse=True)
    w = stream_words(seed, stream, j, _u64(kb)[:, None])
    w = np.stack(np.broadcast_arrays(*w), axis=0)  # [4, len(kb), J]
    q = (k >> 1) & 3
    word = w[q, kb_idx, :]  # [K, J]
    u1 = ((word & M32).astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = ((word >> U64(32)).astype(np.float64) + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    odd = (k & 1).astype(bool)[:, None]
    return np.where(odd, rad * np.sin(ang), rad * np.cos(ang))
