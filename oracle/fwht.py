"""Walsh-Hadamard transform for the oracle (SRHT definition, Sec. 3).

H is the Sylvester-order Hadamard matrix, H_{jk} = (-1)^{popcount(j & k)},
built by H_{2n} = [[H_n, H_n], [H_n, -H_n]], left unnormalised; the paper's
normalised H is H / sqrt(N').  The transform acts along axis 0 of a 2-D array.
"""
import numpy as np


def fwht(v):
    """Unnormalised H @ v along axis 0 (length a power of 2), in float64."""
    z = np.array(v, dtype=np.float64, copy=True)
    n = z.shape[0]
    if n & (n - 1):
        raise ValueError("length must be a power of 2")
    tail = z.shape[1:]
    h = 1
    while h < n:
        z = z.reshape((n // (2 * h), 2, h) + tail)
        a = z[:, 0].copy()
        b = z[:, 1]
        z[:, 0] = a + b
        z[:, 1] = a - b
        z = z.reshape((n,) + tail)
        h *= 2
    return z


def hadamard_dense(n):
    """Dense H_n from the popcount formula (for small n only)."""
    j = np.arange(n)
    bits = np.bitwise_and.outer(j, j)
    pop = np.zeros_like(bits)
    while np.any(bits):
        pop += bits & 1
        bits >>= 1
    return np.where(pop % 2 == 0, 1.0, -1.0)


def hadamard_rows(rows, n, cols=None):
    """Entries H_n[rows, cols] (popcount formula) as a float64 array; all n
    columns when `cols` is None."""
    j = np.asarray(rows, dtype=np.int64)[:, None]
    k = (np.arange(n, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64))[None, :]
    pop = np.bitwise_count(j & k)
    return np.where(pop % 2 == 0, 1.0, -1.0)
