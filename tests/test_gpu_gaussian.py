"""GPU parity of the Gaussian sketch when its data rows are cut into several
splits (each split sums a contiguous range of rows of [X|Y]; a reduction adds
the splits in order), against the oracle's G[X|Y] on the same rounded operands.

Bounds, per output entry (k, c), with T = sum_j |G_kj| |W_jc|:
  * accumulation: every addition of a split's running sum and of the split
    reduction rounds once, so |error| <= (n_add) u T with n_add the additions
    on the longest chain (a split's rows, times 17/16 for the 16-product
    matrix-core steps, plus the number of splits);
  * entries of G: the device draws G in FP32 (libm-style or hardware
    transcendentals) while the oracle draws it in FP64; for the FP32/FP64 form
    they differ by at most delta_kj = 2^-16 (1 + |G_kj|), adding
    sum_j delta_kj |W_jc|; for the BF16 form they round to the same BF16 value
    unless the FP64 value lies within delta_kj of a BF16 rounding midpoint,
    and such entries may differ by one BF16 ulp, adding
    sum_{j uncertain} ulp(G_kj) |W_jc|.
Each case also checks that the bound is tight enough to see a missing chunk
of 64 data rows: the oracle with one chunk left out violates it.
"""
import numpy as np
import pytest
import torch

from oracle import rng as R
from oracle import sketch as S

from bounds import bf16_uncertain

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_06856_amd import slse

    return slse


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _ranges(N, splits, bf16):
    per = -(-N // splits)
    if bf16:
        per = -(-per // 64) * 64
    return [(s * per, min(N, (s + 1) * per)) for s in range(splits) if s * per < N]


def _case(G, N, d, m, r, form, seed=88, drop_rows=64, check_drop=True):
    dtype = {"bf16": np.float32, "f32": np.float32, "f64": np.float64}[form]
    bf16 = form == "bf16"
    splits_a = G.debug_gaussian_plan(N, d, m[-1], bf16)
    splits_h = G.debug_gaussian_plan(N, d, r, bf16)
    g = np.random.default_rng(N + d)
    X = g.standard_normal((N, d)).astype(dtype)
    Y = g.standard_normal(N).astype(dtype)
    A, Ah, _ = G.sketch_apply(dev(X), dev(Y), "gaussian", seed, m, r, bf16=bf16)
    A, Ah = A.cpu().numpy(), Ah.cpu().numpy()
    if bf16:
        W = S.joint(S.round_to(X, "bf16"), S.round_to(Y, "bf16"))
    else:
        W = S.joint(X.astype(np.float64), Y.astype(np.float64))
    u = U64 if form == "f64" else U32
    Wabs = np.abs(W)
    for out, stream, rows, splits in ((A, R.STREAM_G, m[-1], splits_a),
                                      (Ah, R.STREAM_GHAT, r, splits_h)):
        ranges = _ranges(N, splits, bf16)
        longest = max(b - a for a, b in ranges)
        n_add = (longest * 17 // 16 if bf16 else longest) + len(ranges) + 16
        ref = np.zeros((rows, d + 1))
        T = np.zeros((rows, d + 1))
        extra = np.zeros((rows, d + 1))
        drop = np.zeros((rows, d + 1))  # the contribution of one chunk of drop_rows rows
        j_drop = (ranges[-1][0] - drop_rows, ranges[-1][0])
        for j0 in range(0, N, 4096):
            j = np.arange(j0, min(N, j0 + 4096))
            g64 = R.gaussian_block(seed, stream, np.arange(rows), j)
            delta = 2.0 ** -16 * (1.0 + np.abs(g64))
            if bf16:
                gq = S.round_to(g64, "bf16")
                unc, ulp = bf16_uncertain(g64, delta)
                extra += (np.where(unc, ulp, 0.0)) @ Wabs[j]
            else:
                gq = g64
                extra += delta @ Wabs[j]
            ref += gq @ W[j]
            T += np.abs(gq) @ Wabs[j]
            sel = (j >= j_drop[0]) & (j < j_drop[1])
            if sel.any():
                drop += gq[:, sel] @ W[j[sel]]
        tol = n_add * u * T + extra + 1e-300
        err = np.abs(out[:rows, : d + 1] - ref)
        assert np.all(err <= tol), (form, stream, float((err / tol).max()))
        # a missing chunk of rows (just before the last split) would not pass
        if check_drop:
            assert np.any(np.abs(drop) > 2 * tol), (form, stream)
    return splits_a, splits_h


@pytest.mark.parametrize("form", ["bf16", "f32", "f64"])
@pytest.mark.parametrize("d", [37, 512, 700])
def test_gaussian_four_splits_with_a_short_last_split(G, form, d):
    # N = 16400 is not a multiple of 64 x splits: four splits, the last one short
    N = 16400
    sa, sh = _case(G, N, d, [32, 200], 256 if d < 256 else d + 60, form)
    assert sa == 4 and sh == 4


@pytest.mark.slow
@pytest.mark.parametrize("form", ["bf16", "f32"])
def test_gaussian_many_splits(G, form):
    # 2^17 + 37 rows: 25 to 32 splits and a ragged last one; at this length the
    # accumulation bound is checked to exclude a missing split's worth of rows
    N, d = (1 << 17) + 37, 512
    sa, sh = _case(G, N, d, [64, 192], 576, form, seed=91, drop_rows=4096)
    assert sa >= 25 and sh >= 25


@pytest.mark.slow
@pytest.mark.parametrize("form", ["bf16", "f32"])
def test_gaussian_empty_last_split(G, form):
    # 2^19 + 1 rows: 128 splits; in the BF16 form the split length rounds up
    # to whole 64-row steps (4160 rows), so the last split starts past the data
    # and must still write zero partials.  A sketch of the first 2^19 rows,
    # scaled by 1e6, runs first and leaves that split's partials in the
    # context's scratch about 1e7 in size: far above the bound if they were
    # summed again.  (At this length the accumulation bound is too loose to
    # see one missing chunk of rows; the other cases check that.)
    N, d, m, r = (1 << 19) + 1, 16, [32], 40
    bf16 = form == "bf16"
    splits = G.debug_gaussian_plan(N, d, r, bf16)
    assert splits == G.debug_gaussian_plan(N - 1, d, r, bf16) == 128
    if bf16:
        per = -(-(-(-N // splits)) // 64) * 64
        assert (splits - 1) * per >= N
    dtype = np.float32
    g = np.random.default_rng(N + d)
    X = g.standard_normal((N, d)).astype(dtype)
    Y = g.standard_normal(N).astype(dtype)
    G.sketch_apply(dev(1e6 * X[: N - 1]), dev(1e6 * Y[: N - 1]), "gaussian", 93, m, r, bf16=bf16)
    torch.cuda.synchronize()
    _case(G, N, d, m, r, form, seed=88, check_drop=False)
