"""Pins of the oracle's Hadamard transform and sketches (CPU only)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import fwht as F
from oracle import sketch as S
from oracle import rng


@pytest.mark.parametrize("n", [2, 4, 8, 64, 1024])
def test_fwht_equals_dense_popcount_and_scipy(n):
    g = np.random.default_rng(n)
    v = g.standard_normal((n, 3))
    Hd = F.hadamard_dense(n)
    assert np.array_equal(Hd, scipy.linalg.hadamard(n))
    np.testing.assert_allclose(F.fwht(v), Hd @ v, rtol=1e-12, atol=1e-12)


def test_fwht_involution_and_parseval():
    g = np.random.default_rng(1)
    v = g.standard_normal((4096, 5))
    z = F.fwht(v)
    np.testing.assert_allclose(F.fwht(z) / 4096, v, atol=1e-12)
    np.testing.assert_allclose((z ** 2).sum(0), 4096 * (v ** 2).sum(0), rtol=1e-12)


def test_hadamard_rows_matches_dense():
    Hd = F.hadamard_dense(256)
    rows = [0, 1, 77, 255]
    assert np.array_equal(F.hadamard_rows(rows, 256), Hd[rows])


def _problem(n, d, seed=0):
    g = np.random.default_rng(seed)
    return g.standard_normal((n, d)), g.standard_normal(n)


def test_srht_rows_match_transform_with_padding():
    X, Y = _problem(1000, 5)  # pads to 1024
    Z, p = S.srht_transform(X, Y, 31)
    assert p == 10 and Z.shape == (1024, 6)
    rows = [0, 5, 999, 1023]
    np.testing.assert_allclose(S.srht_rows(X, Y, 31, rows), Z[rows], rtol=1e-12, atol=1e-11)


def test_srht_levels_are_prefixes_and_distinct_rows():
    X, Y = _problem(512, 4)
    sk = S.srht(X, Y, 3, [16, 32, 64], 24)
    Z, p = S.srht_transform(X, Y, 3)
    sigma, sigma_hat = S.srht_orders(3, p, 64, 24)
    assert len(np.unique(sigma)) == 64
    np.testing.assert_array_equal(sk["A"], Z[sigma])
    np.testing.assert_array_equal(sk["Ahat"], Z[sigma_hat])
    assert sk["scale"] == [1 / 16, 1 / 32, 1 / 64] and sk["hat_scale"] == 1 / 24


def test_srht_full_sample_is_orthogonal():
    # with every row kept, S = H_norm D P is orthogonal: (1/N') A^T A = W^T W
    X, Y = _problem(256, 6)
    sk = S.srht(X, Y, 8, [256], 256)
    W = S.joint(X, Y)
    np.testing.assert_allclose(sk["A"].T @ sk["A"] / 256, W.T @ W, rtol=1e-11, atol=1e-10)


@pytest.mark.parametrize("kind", ["srht", "countsketch", "gaussian"])
def test_sketch_is_unbiased(kind):
    # E[c_i A_i^T A_i] = [X|Y]^T [X|Y] (E[S^T S] = I), Monte Carlo over seeds
    X, Y = _problem(64, 3, seed=2)
    W = S.joint(X, Y)
    acc = np.zeros((4, 4))
    reps = 300 if kind != "gaussian" else 150
    for seed in range(reps):
        sk = S.sketch(kind, X, Y, seed, [8, 16], 12)
        A = sk["A"][sk["offset"][0]: sk["offset"][0] + 8]
        acc += sk["scale"][0] * A.T @ A
    est = acc / reps
    rel = np.linalg.norm(est - W.T @ W) / np.linalg.norm(W.T @ W)
    assert rel < 0.12


def test_srht_subspace_embedding_near_mp_edge():
    # Definition 3.1 with Thm 3.2's SRHT: ||U^T S^T S U - I|| is O(sqrt(d/m))
    X, Y = _problem(4096, 8, seed=5)
    U, _ = np.linalg.qr(np.concatenate([X, Y[:, None]], axis=1))
    sk = S.srht(U[:, :-1], U[:, -1], 7, [512], 128)
    SU = sk["A"] / np.sqrt(512)
    eps = np.linalg.norm(SU.T @ SU - np.eye(9), 2)
    edge = 2 * np.sqrt(9 / 512) + 9 / 512
    assert eps < 2.0 * edge


def test_countsketch_levels_fold():
    X, Y = _problem(3000, 4, seed=3)
    sk = S.countsketch(X, Y, 9, [32, 64, 128], 40)
    A1 = sk["A"][0:32]
    A2 = sk["A"][32:96]
    A3 = sk["A"][96:224]
    np.testing.assert_allclose(A2[:32] + A2[32:], A1, atol=1e-12)
    np.testing.assert_allclose(A3[:64] + A3[64:], A2, atol=1e-12)
    # brute force of level 1 from its definition
    h, s = rng.countsketch_hash(9, 3000, 128)
    W = S.joint(X, Y)
    ref = np.zeros((32, 5))
    for j in range(3000):
        ref[h[j] % 32] += s[j] * W[j]
    np.testing.assert_allclose(A1, ref, atol=1e-11)


def test_gaussian_sketch_blockwise_equals_dense():
    X, Y = _problem(300, 3, seed=4)
    sk = S.gaussian(X, Y, 5, [8, 16], 10)
    G = rng.gaussian_block(5, rng.STREAM_G, np.arange(16), np.arange(300))
    np.testing.assert_allclose(sk["A"], G @ S.joint(X, Y), rtol=1e-12, atol=1e-12)


def test_round_to_bf16_and_f32():
    a = np.array([1.0, 1.00390625, 1.005859375, -3.1415926, 1e-20])
    b = S.round_to(a, "bf16")
    # bf16 keeps 8 significant bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-9 -> 1 + 2^-7
    assert b[0] == 1.0 and b[1] == 1.0 and b[2] == 1.0078125
    assert abs(b[3] + 3.140625) < 1e-12
    assert S.round_to(a, "f32")[3] == np.float32(-3.1415926)
