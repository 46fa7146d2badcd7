"""Rounding-bound helpers shared by the GPU parity tests (no GPU needed)."""
import numpy as np


def bf16_uncertain(g64, delta):
    """Entries whose FP64 value lies within delta of a BF16 rounding midpoint
    (so that a value off by up to delta may round to the neighbouring BF16
    number), and the BF16 ulp at each entry."""
    f = g64.astype(np.float32)
    u = f.view(np.uint32)
    lo = (u & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    mid = (u & np.uint32(0xFFFF0000) | np.uint32(0x8000)).view(np.float32).astype(np.float64)
    hi_bits = (u & np.uint32(0xFFFF0000)) + np.uint32(0x10000)
    ulp = np.abs(hi_bits.view(np.float32).astype(np.float64) - lo)
    return np.abs(np.abs(g64) - np.abs(mid)) <= delta, ulp
