"""Pins of the oracle's counter-based randomness (CPU only).

Philox4x64-10 is checked against NumPy's independent Philox bit generator
(which increments its counter before each block).  The keyed permutation is
checked to be a bijection by brute force, the inverse to round-trip, and the
signs, hashes and Gaussians against their distributions.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import rng


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 12345), (1009, 3)])
def test_philox_matches_numpy_bit_generator(key):
    ctr = np.array([2**64 - 3, 17, 2**63, 1], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=ctr)
    ref = bg.random_raw(4 * 6).reshape(6, 4)
    for b in range(6):
        # numpy increments the 256-bit counter (word 0 first, with carry) before use
        c0 = (int(ctr[0]) + b + 1) % 2**64
        carry = (int(ctr[0]) + b + 1) // 2**64
        c1 = int(ctr[1]) + carry
        out = rng.philox4x64(np.uint64(c0), np.uint64(c1), ctr[2], ctr[3], key[0], key[1])
        assert [int(x) for x in out] == [int(x) for x in ref[b]]


def test_philox_vectorised_equals_scalar():
    c = np.arange(100, dtype=np.uint64) * np.uint64(7919)
    vec = rng.philox4x64(c, 3, 0, 0, 11, 4)
    for i in (0, 1, 50, 99):
        sc = rng.philox4x64(c[i], 3, 0, 0, 11, 4)
        assert all(int(vec[w][i]) == int(sc[w]) for w in range(4))


@pytest.mark.parametrize("p", list(range(1, 17)))
def test_prp_is_bijection_and_inverse(p):
    n = 1 << p
    x = np.arange(n)
    for stream in (rng.STREAM_P, rng.STREAM_S):
        y = rng.prp(x, 77, stream, p)
        assert y.max() < n
        assert len(np.unique(y)) == n
        assert np.array_equal(rng.prp_inverse(y, 77, stream, p), x.astype(np.uint64))


@pytest.mark.slow
@pytest.mark.parametrize("p", [19, 20])
def test_prp_bijection_large(p):
    n = 1 << p
    y = rng.prp(np.arange(n), 5, rng.STREAM_SHAT, p)
    assert len(np.unique(y)) == n


def test_prp_depends_on_seed_and_stream():
    x = np.arange(1024)
    a = rng.prp(x, 1, rng.STREAM_S, 10)
    b = rng.prp(x, 2, rng.STREAM_S, 10)
    c = rng.prp(x, 1, rng.STREAM_SHAT, 10)
    assert not np.array_equal(a, b)
    assert not np.array_equal(a, c)
    # not the identity, and no long fixed runs
    assert np.mean(a == x) < 0.01


def test_prp_positions_uniform():
    # where does element 0 land over many keys: roughly uniform over 16 slots
    p = 4
    hits = np.zeros(16)
    for seed in range(3000):
        hits[int(rng.prp(np.array([0]), seed, rng.STREAM_P, p)[0])] += 1
    chi2 = ((hits - hits.mean()) ** 2 / hits.mean()).sum()
    assert chi2 < stats.chi2.ppf(0.999, 15)


def test_rademacher_balanced_and_blocked():
    D = rng.rademacher(9, 1 << 16)
    assert set(np.unique(D)) == {-1, 1}
    assert abs(D.mean()) < 4 / np.sqrt(D.size)
    # the first 300 signs equal the prefix of a longer draw (index-addressable)
    assert np.array_equal(rng.rademacher(9, 300), D[:300])
    # lag-1 correlation is small
    assert abs(np.mean(D[1:] * D[:-1])) < 4 / np.sqrt(D.size)


def test_countsketch_hash_ranges_and_uniformity():
    h, s = rng.countsketch_hash(3, 1 << 16, 256)
    assert h.min() >= 0 and h.max() < 256
    counts = np.bincount(h, minlength=256)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert chi2 < stats.chi2.ppf(0.999, 255)
    assert abs(s.astype(float).mean()) < 4 / np.sqrt(s.size)
    hh, ss = rng.countsketch_hash_hat(3, 1 << 16, 192)
    assert hh.min() >= 0 and hh.max() < 192
    counts = np.bincount(hh, minlength=192)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert chi2 < stats.chi2.ppf(0.999, 191)


def test_gaussian_distribution():
    G = rng.gaussian_block(4, rng.STREAM_G, np.arange(64), np.arange(4096)).ravel()
    assert stats.kstest(G, "norm").pvalue > 1e-3
    assert abs(G.mean()) < 5 / np.sqrt(G.size)
    assert abs(G.var() - 1) < 5 * np.sqrt(2 / G.size)
    # the cosine and sine halves of one Box-Muller pair are uncorrelated
    B = rng.gaussian_block(4, rng.STREAM_G, np.arange(8), np.arange(20000))
    assert abs(np.corrcoef(B[0], B[1])[0, 1]) < 0.05


def test_gaussian_entry_is_index_addressable():
    full = rng.gaussian_block(8, rng.STREAM_GHAT, np.arange(24), np.arange(50))
    part = rng.gaussian_block(8, rng.STREAM_GHAT, np.array([3, 17, 23]), np.array([0, 49]))
    assert np.array_equal(part, full[np.ix_([3, 17, 23], [0, 49])])
