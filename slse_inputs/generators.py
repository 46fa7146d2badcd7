"""Synthetic linear models Y = X beta + zeta shaped like the paper's workloads.

The paper builds X = G D with G an iid Gaussian N x d matrix and D a diagonal
column scaling that sets the condition number, beta iid N(0, 1) and zeta iid
N(0, sigma^2) (Sec. 5, the test-problem generator).  The named workloads below
follow that recipe with the sizes, conditioning, leverage and noise of the
regressions this library is measured on:

  plain_small     N=16384,  d=32,  X iid N(0,1), sigma=1e-2, float64
  illcond         N=2^20,   d=256, X = G diag(s) V^T, s log-spaced 1..1e-4,
                  V a seeded random orthogonal matrix (a Givens butterfly network,
                  not Haar distributed), 5% of rows scaled x100, sigma=1e-3, float64
  mixed           N=2^22,   d=512, X = G diag(s), s log-spaced 1..1e-6,
                  sigma=1e-2, X and Y rounded to float32
  backward        N=2^20,   d=256, X iid N(0,1), sigma=1e-2, float32, plus a
                  loss vector w iid N(0,1)
  batched         64 problems, N_b uniform on [2^14, 2^18], d_b uniform on
                  {16, 32, 64, 128, 256}, rows multivariate Student-t(3),
                  columns scaled to unit norm, sigma=1e-2, float32

Random numbers come from numpy.random.Generator(Philox(key=(seed, block))),
one generator per block of 2^16 rows, so blocks can be drawn in parallel and
the result does not depend on the thread count.  Everything after the draws
is elementwise IEEE arithmetic in a fixed order (no BLAS, no vectorised libm),
so a workload regenerates bit for bit on any x86-64 host with this NumPy and
glibc; `fingerprint()` hashes the arrays to check that.  The orthogonal V of
the ill-conditioned workload is a random butterfly network of Givens
rotations (three sweeps over the pairs (i, i xor 2^l)), applied row by row.
A smaller `n` (and `d`) may be requested for any workload to get a
same-recipe problem of another size.
"""
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
import math
import os

import numpy as np

DATA_SEED_BASE = 2509068560
ROW_BLOCK = 1 << 16

WORKLOADS = {
    "plain_small": dict(k=1, n=16384, d=32, dtype="float64"),
    "illcond": dict(k=2, n=1 << 20, d=256, dtype="float64"),
    "mixed": dict(k=3, n=1 << 22, d=512, dtype="float32"),
    "backward": dict(k=4, n=1 << 20, d=256, dtype="float32"),
    "batched": dict(k=5, n=None, d=None, dtype="float32"),
}


def sketch_seed(name, rep=0):
    """Sketch seed of a workload: 1000 + k (+ 100 per repetition)."""
    return 1000 + WORKLOADS[name]["k"] + 100 * rep


@dataclass
class Problem:
    name: str
    X: np.ndarray
    Y: np.ndarray
    beta_true: np.ndarray
    sigma: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]


def _gen(seed, block):
    return np.random.Generator(np.random.Philox(key=np.array([seed, block], dtype=np.uint64)))


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _fill_blocks(n, fn):
    blocks = list(range((n + ROW_BLOCK - 1) // ROW_BLOCK))
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fn, blocks))


def _logspace_scale(d, smin):
    """s_k = smin^(k/(d-1)), k = 0..d-1 (scalar libm calls, so bit-reproducible)."""
    if d == 1:
        return np.ones(1)
    e = math.log10(smin)
    return np.array([math.pow(10.0, e * k / (d - 1)) for k in range(d)])


def _rotation_network(d, rng, sweeps=3):
    """Layers of Givens rotations (i, i ^ 2^l) with random angles: a random orthogonal V."""
    layers = []
    for _ in range(sweeps):
        l = 1
        while l < d:
            i = np.array([k for k in range(d) if (k & l) == 0 and (k | l) < d], dtype=np.int64)
            theta = rng.uniform(0.0, 2.0 * math.pi, size=len(i))
            c = np.array([math.cos(t) for t in theta])
            s = np.array([math.sin(t) for t in theta])
            layers.append((i, i | l, c, s))
            l <<= 1
    return layers


def _apply_rotations(Xb, layers):
    """Xb <- Xb V^T, one rotation layer at a time (elementwise, fixed order)."""
    for i, j, c, s in layers:
        xi = Xb[:, i]
        xj = Xb[:, j]
        Xb[:, i] = xi * c - xj * s
        Xb[:, j] = xi * s + xj * c
    return Xb


def _matvec(Xb, beta):
    """Xb @ beta as a fixed-order sum over columns (no BLAS)."""
    y = np.zeros(Xb.shape[0])
    for k in range(Xb.shape[1]):
        y += Xb[:, k] * beta[k]
    return y


def fingerprint(*arrays):
    """xxh64 of the arrays' bytes, to check that a workload regenerated bit for bit."""
    import xxhash

    h = xxhash.xxh64()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def make_problem(name, n=None, d=None, seed=None):
    """Generate workload `name` (optionally at another size)."""
    spec = WORKLOADS[name]
    if name == "batched":
        raise ValueError("use make_batched()")
    n = spec["n"] if n is None else int(n)
    d = spec["d"] if d is None else int(d)
    seed = DATA_SEED_BASE + spec["k"] if seed is None else int(seed)
    out_dtype = np.dtype(spec["dtype"])
    head = _gen(seed, 1 << 40)
    beta = head.standard_normal(d)
    meta = dict(seed=seed, dtype=out_dtype.name)

    if name in ("plain_small", "backward"):
        sigma = 1e-2
        scale = np.ones(d)
        V = None
        lev = None
    elif name == "illcond":
        sigma = 1e-3
        scale = _logspace_scale(d, 1e-4)
        V = _rotation_network(d, head)
        k_lev = int(round(0.05 * n))
        lev = np.zeros(n, dtype=bool)
        lev[head.permutation(n)[:k_lev]] = True
        meta["leverage_rows"] = k_lev
    elif name == "mixed":
        sigma = 1e-2
        scale = _logspace_scale(d, 1e-6)
        V = None
        lev = None
    else:
        raise ValueError(name)

    X = np.empty((n, d), dtype=out_dtype)
    Y = np.empty(n, dtype=out_dtype)

    def block(b):
        g = _gen(seed, b)
        i0 = b * ROW_BLOCK
        i1 = min(n, i0 + ROW_BLOCK)
        G = g.standard_normal((i1 - i0, d))
        Xb = np.asfortranarray(G * scale[None, :])  # columns contiguous for the loops below
        if V is not None:
            Xb = _apply_rotations(Xb, V)
        if lev is not None:
            Xb[lev[i0:i1]] *= 100.0
        zeta = sigma * g.standard_normal(i1 - i0)
        X[i0:i1] = Xb.astype(out_dtype)
        Y[i0:i1] = (_matvec(Xb, beta) + zeta).astype(out_dtype)

    _fill_blocks(n, block)
    meta["scale_min"] = float(scale.min())
    return Problem(name, X, Y, beta, sigma, meta)


def loss_vector(d, seed=None):
    """w iid N(0,1) for the backward workload's loss L = w^T beta_hat."""
    seed = DATA_SEED_BASE + WORKLOADS["backward"]["k"] if seed is None else seed
    return _gen(seed, (1 << 40) + 1).standard_normal(d)


def batched_shapes(count=64, seed=None, n_range=(1 << 14, 1 << 18), d_choices=(16, 32, 64, 128, 256)):
    """The (N_b, d_b) of the batched workload, drawn without generating the data."""
    seed = DATA_SEED_BASE + WORKLOADS["batched"]["k"] if seed is None else int(seed)
    head = _gen(seed, 1 << 40)
    ns = head.integers(n_range[0], n_range[1], endpoint=True, size=count)
    ds = head.choice(np.asarray(d_choices), size=count)
    return [(int(n), int(d)) for n, d in zip(ns, ds)]


def make_batched(count=64, seed=None, n_range=(1 << 14, 1 << 18), d_choices=(16, 32, 64, 128, 256)):
    """The batched workload: `count` independent float32 problems."""
    seed = DATA_SEED_BASE + WORKLOADS["batched"]["k"] if seed is None else int(seed)
    shapes = batched_shapes(count, seed, n_range, d_choices)
    ns = [n for n, _ in shapes]
    ds = [d for _, d in shapes]
    probs = []
    for b in range(count):
        g = _gen(seed, b)
        n, d = int(ns[b]), int(ds[b])
        z = g.standard_normal((n, d))
        w = g.chisquare(3, size=n)
        Xb = np.asfortranarray(z / np.sqrt(w / 3.0)[:, None])
        Xb /= np.sqrt(np.add.reduce(Xb * Xb, axis=0))[None, :]
        beta = g.standard_normal(d)
        sigma = 1e-2
        Y = _matvec(Xb, beta) + sigma * g.standard_normal(n)
        probs.append(Problem("batched", np.ascontiguousarray(Xb, dtype=np.float32),
                             Y.astype(np.float32), beta, sigma, dict(seed=seed, index=b)))
    return probs


def paper_problem(n, d, kappa, sigma2=1e-8, seed=DATA_SEED_BASE + 100, dtype=np.float64):
    """The paper's own recipe: X = G D, D log-spaced 1..1/kappa, zeta ~ N(0, sigma2)."""
    head = _gen(seed, 1 << 40)
    beta = head.standard_normal(d)
    scale = _logspace_scale(d, 1.0 / kappa)
    sigma = float(np.sqrt(sigma2))
    X = np.empty((n, d), dtype=dtype)
    Y = np.empty(n, dtype=dtype)

    def block(b):
        g = _gen(seed, b)
        i0 = b * ROW_BLOCK
        i1 = min(n, i0 + ROW_BLOCK)
        Xb = np.asfortranarray(g.standard_normal((i1 - i0, d)) * scale[None, :])
        X[i0:i1] = Xb
        Y[i0:i1] = _matvec(Xb, beta) + sigma * g.standard_normal(i1 - i0)

    _fill_blocks(n, block)
    return Problem("paper", X, Y, beta, sigma, dict(seed=seed, kappa=kappa))
