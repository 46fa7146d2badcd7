"""Host-only entry points of the C ABI, checked on the CPU (no device work).

* slse_paper_schedule / slse_paper_params / slse_stage1_counts against the
  oracle's schedule, step sizes and real-valued bound of Thm lowerBoundai;
* slse_debug_batch_plan: the batched solve's whole host plan (pools,
  offsets, SRHT job and record tables, factor jobs, per-step tile tables)
  built on a measuring arena and bounds-checked, for the batched workload's
  64 problems, for its 6-problem sample and for mixed sketch kinds.
"""
import math

import pytest
import torch

from oracle import slse as OS
from paper_2509_06856_amd import _lib as L
from paper_2509_06856_amd import slse as G
from slse_inputs import batched_shapes


@pytest.mark.parametrize("n,d", [(1 << 20, 64), (1 << 22, 512), (1 << 20, 256), (100000, 70),
                                 (16384, 32), (1 << 18, 64), (1 << 20, 1024), (70000, 5),
                                 (4096, 1), (3 << 20, 100)])
def test_paper_schedule_matches_oracle(n, d):
    assert G.paper_schedule(n, d) == OS.paper_schedule(n, d)
    assert G.paper_schedule(n, d, m1_factor=2) == OS.paper_schedule(n, d, m1_factor=2)


def test_paper_schedule_errors():
    assert OS.paper_schedule(1000, 100) == []
    with pytest.raises(L.SlseError):
        G.paper_schedule(1000, 100)  # empty schedule
    with pytest.raises(L.SlseError):
        G.paper_schedule(10, 10)     # N <= d


@pytest.mark.parametrize("d", [1, 7, 32, 64, 256, 512, 1024])
def test_paper_params_match_oracle(d):
    r, mu, eta = G.paper_params(d)
    assert r == 6 * d
    mu_o, eta_o = OS.default_params(d, r)
    assert (mu, eta) == (mu_o, eta_o)
    r2, mu2, eta2 = G.paper_params(d, 10 * d)
    assert r2 == 10 * d and (mu2, eta2) == OS.default_params(d, 10 * d)
    with pytest.raises(L.SlseError):
        G.paper_params(d, d)


@pytest.mark.parametrize("omega", [1 / 16, 1 / 8, 1 / 4, 1 / 2, 1.0])
def test_stage1_counts_are_the_ceiling_of_the_oracle_bound(omega):
    for n, d in ((1 << 20, 64), (1 << 22, 512), (100000, 70)):
        m = OS.paper_schedule(n, d)
        lb = OS.iteration_lower_bounds(m, d, omega)
        a = G.auto_a(m, d, omega, a1=5)
        assert a[0] == 5
        assert a[1:] == [max(1, math.ceil(x - 1e-12)) for x in lb[1:]]
        assert G.auto_a(m, d, omega)[0] == a[1]  # a_1 defaults to a_2
    assert G.auto_a([512], 64, 0.5) == [2]


def _batch_params(shapes, kinds=None, factor="chol", precision="mixed"):
    out = []
    for i, (n, d) in enumerate(shapes):
        m = OS.paper_schedule(n, d)
        kind = kinds[i % len(kinds)] if kinds else "srht"
        out.append(G.Params(kind=kind, seed=2000 + i, m=m, a=[2] * len(m), r=6 * d, s_max=45,
                            precision=precision, factor=factor))
    return out


def test_batch_plan_of_the_batched_workload():
    shapes = batched_shapes()
    assert len(shapes) == 64
    need = G.debug_batch_plan(shapes, _batch_params(shapes))
    # the pools hold at least the sketch rows and the Hessian sketches
    rows = sum(OS.paper_schedule(n, d)[-1] * (d + 1) + 6 * d * (d + 1) for n, d in shapes)
    assert need >= 4 * rows


def test_batch_plan_of_the_sample_that_was_skipped_on_the_gpu():
    shapes = batched_shapes(count=6, n_range=(1 << 14, 1 << 15))
    assert shapes[0] == (31242, 128)
    G.debug_batch_plan(shapes, _batch_params(shapes))


@pytest.mark.parametrize("kinds,factor,dtype", [
    (["srht", "countsketch", "gaussian"], "chol", torch.float32),
    (["srht", "countsketch"], "qr", torch.float32),
    (["srht"], "chol", torch.float64),
])
def test_batch_plan_mixed_kinds(kinds, factor, dtype):
    shapes = [(900, 8), (3000, 12), (6000, 16), (11000, 8), (2500, 10), (1800, 6), (40000, 40),
              (17000, 100), (5000, 5), (70000, 32)]
    prec = "mixed" if dtype == torch.float32 else "f64"
    G.debug_batch_plan(shapes, _batch_params(shapes, kinds, factor, prec), dtype=dtype)
