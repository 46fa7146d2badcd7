"""The library's counter-based streams at scale (GPU, bit-exact).

* 10^8 Philox4x64-10 counters (four 64-bit words each) against NumPy's own
  Philox bit generator, an implementation independent of both the library and
  the oracle, in chunks that start at random counters and across a carry of
  the low 32-bit half of the counter word.
* The keyed permutation over every power-of-2 domain 2^1 .. 2^22 in full for
  the permutation stream P (odd p walk cycles over the 2^(p+1)-point Feistel
  domain), and over every domain up to 2^20 for the two sample orders; the
  inverse is checked to undo the forward map on the whole domain.
"""
import numpy as np
import pytest
import torch

from oracle import rng as R

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_06856_amd import slse

    return slse


def test_philox_1e8_counters_against_numpy(G):
    seed, stream, aux = 0x0123456789ABCDEF, 9, 5
    chunk = 25_000_000
    starts = [0, (1 << 32) - chunk // 2, 7_777_777_777_777, (1 << 61) + 12345]
    total = 0
    for start in starts:
        out = G.debug_stream(0, seed, stream, aux, start, chunk).cpu().numpy().view(np.uint64)
        # NumPy's Philox increments its 256-bit counter before each block
        bg = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64),
                              counter=np.array([start - 1 if start else 2**64 - 1,
                                                aux if start else aux - 1, 0, 0], dtype=np.uint64))
        ref = bg.random_raw(4 * chunk)
        assert np.array_equal(out, ref), start
        total += chunk
        del out, ref
    assert total >= 10 ** 8


@pytest.mark.parametrize("p", list(range(1, 23)))
def test_permutation_every_domain(G, p):
    n = 1 << p
    x = np.arange(n)
    streams = [R.STREAM_P] + ([R.STREAM_S, R.STREAM_SHAT] if p <= 20 else [])
    for stream in streams:
        fwd = G.debug_stream(1, 4242, stream, p, 0, n).cpu().numpy()
        assert np.array_equal(fwd, R.prp(x, 4242, stream, p).astype(np.int64)), (p, stream)
        inv = G.debug_stream(2, 4242, stream, p, 0, n).cpu().numpy()
        assert np.array_equal(inv[fwd], x), (p, stream)
