"""Host logic of the batched solve: how one step's rows are cut into tiles
(slse_debug_batch_tiles runs the library's own split on the host; no GPU)."""
import ctypes
import os

import numpy as np
import pytest


@pytest.fixture(scope="module")
def lib():
    from paper_2509_06856_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libslse.so not built")
    return _lib.load()


def split(lib, n, row_bytes, step_rows, slots, min_tile):
    B = len(n)
    a = lambda v: np.ascontiguousarray(v, dtype=np.int64)
    n, rb, sr = a(n), a(row_bytes), a(step_rows)
    tr = np.zeros(B, dtype=np.int32)
    nt = np.zeros(B, dtype=np.int32)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    st = lib.slse_debug_batch_tiles(B, p(n), p(rb), p(sr), slots, min_tile, p(tr), p(nt))
    assert st == 0
    return tr.astype(np.int64), nt.astype(np.int64)


def check_invariants(n, row_bytes, step_rows, tr, nt):
    for b in range(len(n)):
        if n[b] == 0:
            assert nt[b] == 0
            continue
        assert nt[b] >= 1
        assert tr[b] * nt[b] >= n[b]                       # every row is in a tile
        assert (nt[b] - 1) * tr[b] < n[b]                  # no empty tile
        assert nt[b] <= -(-n[b] // 256)                    # the partial pool holds ceil(n / 256)
        assert tr[b] % step_rows[b] == 0 or tr[b] == n[b]  # whole main-loop steps


def test_batch_of_equal_problems_gets_equal_tiles(lib):
    n = [100000] * 8
    rb = [68 * 4] * 8
    sr = [128] * 8
    tr, nt = split(lib, n, rb, sr, slots=1024, min_tile=128 << 10)
    check_invariants(n, rb, sr, tr, nt)
    assert len(set(nt.tolist())) == 1 and len(set(tr.tolist())) == 1
    assert nt.sum() <= 1024


def test_random_batches_keep_the_invariants_and_the_balance(lib):
    g = np.random.default_rng(11)
    for trial in range(40):
        B = int(g.integers(1, 80))
        n = g.integers(1 << 10, 1 << 18, size=B)
        n[g.random(B) < 0.2] = 0                      # idle problems
        d = g.choice([5, 16, 32, 64, 128, 256], size=B)
        rb = (d + 1) * 4
        sr = g.choice([32, 64, 128, 512], size=B)
        slots = int(g.choice([256, 512, 768, 1024, 2048]))
        tr, nt = split(lib, n, rb, sr, slots, 128 << 10)
        check_invariants(n, rb, sr, tr, nt)
        total = float((n * rb).sum())
        if total == 0:
            assert nt.sum() == 0
            continue
        want = min(slots, int(np.ceil(total / (128 << 10))))
        active = int((n > 0).sum())
        # about `want` tiles: the one-tile minimum of small problems and the
        # caps may move the count a little
        assert nt.sum() <= max(want, active) + active
        # problems with many tiles get tiles near the common size
        target = total / max(want, 1)
        for b in range(B):
            if nt[b] >= 8:
                size = tr[b] * rb[b]
                assert 0.5 * target <= size <= 1.5 * target + sr[b] * rb[b], (trial, b)


def test_small_steps_and_tiny_problems(lib):
    # one short problem, one below the 256-row floor, one idle
    n = [9000, 200, 0]
    rb = [17 * 4, 9 * 8, 65 * 4]
    sr = [512, 64, 128]
    tr, nt = split(lib, n, rb, sr, slots=1024, min_tile=128 << 10)
    check_invariants(n, rb, sr, tr, nt)
    assert nt.tolist()[1:] == [1, 0] and tr[1] == 200


def test_bad_arguments_are_rejected(lib):
    from paper_2509_06856_amd import _lib

    B = 2
    n = np.array([10, 10], dtype=np.int64)
    rb = np.array([0, 8], dtype=np.int64)
    sr = np.array([1, 1], dtype=np.int64)
    out = np.zeros(B, dtype=np.int32)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    assert lib.slse_debug_batch_tiles(B, p(n), p(rb), p(sr), 16, 1024, p(out), p(out)) == _lib.SLSE_EINVAL
    assert lib.slse_debug_batch_tiles(B, None, p(rb), p(sr), 16, 1024, p(out), p(out)) == _lib.SLSE_EINVAL
