"""Failure paths of the C ABI, forced from the host (every kernel still exits normally)."""
import ctypes

import numpy as np
import pytest
import torch

from slse_inputs import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_06856_amd import slse

    return slse


@pytest.fixture(scope="module")
def L():
    from paper_2509_06856_amd import _lib

    return _lib


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _small(G, precision="f64", **kw):
    p = make_problem("plain_small", n=4096, d=8)
    prm = G.Params(kind="srht", seed=3, m=[64, 128, 256], a=[2, 2, 2], r=48, s_max=20,
                   precision=precision, **kw)
    return p, prm


def test_null_and_bad_arguments(G, L):
    lib = L.load()
    ctx = G.default_context(0)
    # null problem / params
    st = lib.slse_solve(ctx.h, None, None, None, None, None)
    assert st == L.SLSE_EINVAL and b"null" in lib.slse_last_error()
    # resid grad with ldx < d
    X = torch.zeros((10, 4), dtype=torch.float64, device="cuda:0")
    b = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    g = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    st = lib.slse_fused_resid_grad(ctx.h, 10, 4, ctypes.c_void_p(X.data_ptr()), 3, None,
                                   L.SLSE_F64, ctypes.c_void_p(b.data_ptr()), 1.0, L.SLSE_F64,
                                   ctypes.c_void_p(g.data_ptr()), None, None)
    assert st == L.SLSE_EINVAL
    # unsupported dtype
    st = lib.slse_fused_resid_grad(ctx.h, 10, 4, ctypes.c_void_p(X.data_ptr()), 4, None,
                                   L.SLSE_BF16, ctypes.c_void_p(b.data_ptr()), 1.0, L.SLSE_F64,
                                   ctypes.c_void_p(g.data_ptr()), None, None)
    assert st == L.SLSE_EINVAL


def test_shape_and_schedule_checks(G, L):
    p, prm = _small(G)
    X, Y = dev(p.X), dev(p.Y)
    with pytest.raises(L.SlseError) as e:  # m not increasing
        G.solve(X, Y, G.Params(kind="srht", seed=1, m=[128, 64], a=[1, 1], r=48, s_max=2))
    assert e.value.status == L.SLSE_EINVAL
    with pytest.raises(L.SlseError) as e:  # r <= d
        G.solve(X, Y, G.Params(kind="srht", seed=1, m=[64], a=[1], r=8, s_max=2))
    assert e.value.status == L.SLSE_EINVAL
    with pytest.raises(L.SlseError) as e:  # N <= d
        G.solve(X[:8], Y[:8], G.Params(kind="srht", seed=1, m=[4], a=[1], r=9, s_max=2))
    assert e.value.status == L.SLSE_EINVAL
    with pytest.raises(L.SlseError) as e:  # CountSketch sizes must be powers of 2
        G.solve(X, Y, G.Params(kind="countsketch", seed=1, m=[96], a=[1], r=48, s_max=2))
    assert e.value.status == L.SLSE_EINVAL
    with pytest.raises(L.SlseError) as e:  # precision / dtype mismatch
        G.solve(X, Y, G.Params(kind="srht", seed=1, m=[64], a=[1], r=48, s_max=2,
                               precision="mixed"))
    assert e.value.status == L.SLSE_EINVAL


def test_rank_deficient_sketch_is_singular(G, L):
    p, prm = _small(G)
    Xz = p.X.copy()
    Xz[:, 5] = 0.0
    with pytest.raises(L.SlseError) as e:
        G.solve(dev(Xz), dev(p.Y), prm)
    assert e.value.status == L.SLSE_ESINGULAR


def test_nan_in_data_is_nonfinite(G, L):
    p, prm = _small(G)
    Xn = p.X.copy()
    Xn[1234, 3] = np.nan
    with pytest.raises(L.SlseError) as e:
        G.solve(dev(Xn), dev(p.Y), prm)
    assert e.value.status in (L.SLSE_ENONFINITE, L.SLSE_ESINGULAR)


def test_tolerance_not_met_reports_enotconv_with_last_iterate(G, L):
    p, prm = _small(G, tol=1e-15)
    prm.s_max = 3
    beta, info = G.solve(dev(p.X), dev(p.Y), prm)
    assert info["status"] == "SLSE_ENOTCONV"
    assert torch.isfinite(beta).all()


def test_context_lifecycle(G, L):
    c = G.Context(0)
    p, prm = _small(G)
    b1, _ = G.solve(dev(p.X), dev(p.Y), prm, ctx=c)
    c.trim()
    b2, _ = G.solve(dev(p.X), dev(p.Y), prm, ctx=c)
    assert torch.equal(b1, b2)
    c.close()
    c.close()  # idempotent


def test_batched_argument_checks(G, L):
    # host-side checks before any launch: one storage dtype per batch,
    # d <= 512, and d <= 256 when some rows are not 16-byte aligned
    p = make_problem("plain_small", n=4096, d=8)
    X, Y = dev(p.X), dev(p.Y)
    prm64 = G.Params(kind="srht", seed=1, m=[64, 128], a=[1, 1], r=48, s_max=2)
    prm32 = G.Params(kind="srht", seed=1, m=[64, 128], a=[1, 1], r=48, s_max=2, precision="mixed")
    with pytest.raises(L.SlseError) as e:
        G.solve_batched([X, X.float()], [Y, Y.float()], [prm64, prm32])
    assert e.value.status == L.SLSE_EINVAL and "dtype" in str(e.value)
    Xw = torch.zeros((8192, 520), dtype=torch.float64, device="cuda:0")
    Yw = torch.zeros(8192, dtype=torch.float64, device="cuda:0")
    wide = G.Params(kind="srht", seed=1, m=[4096], a=[1], r=3120, s_max=2)
    with pytest.raises(L.SlseError) as e:
        G.solve_batched([Xw], [Yw], [wide])
    assert e.value.status == L.SLSE_EINVAL and "512" in str(e.value)
    Xu = torch.zeros((4096, 301), dtype=torch.float32, device="cuda:0")  # 1204-byte rows
    Yu = torch.zeros(4096, dtype=torch.float32, device="cuda:0")
    unaligned = G.Params(kind="srht", seed=1, m=[2048], a=[1], r=1806, s_max=2, precision="mixed")
    with pytest.raises(L.SlseError) as e:
        G.solve_batched([Xu], [Yu], [unaligned])
    assert e.value.status == L.SLSE_EINVAL and "too large" in str(e.value)
