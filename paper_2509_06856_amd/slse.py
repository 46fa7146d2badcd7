"""PyTorch-facing wrappers of libslse (names follow include/slse.h).

Tensors supply device memory and the current HIP stream; each call forwards
pointers and sizes to the C ABI and nothing else: the sketch, the factor, the
M-IHS iteration and the adjoint all run in the library's kernels.
"""
import ctypes
from dataclasses import dataclass, field
from typing import List, Optional

import torch

from . import _lib as L

_DT = {torch.float32: L.SLSE_F32, torch.float64: L.SLSE_F64}
_KIND = {"srht": L.SLSE_SRHT, "countsketch": L.SLSE_COUNTSKETCH, "gaussian": L.SLSE_GAUSSIAN}
_FACTOR = {"chol": L.SLSE_FACTOR_CHOL, "qr": L.SLSE_FACTOR_QR}
_PREC = {"f64": L.SLSE_PREC_F64, "mixed": L.SLSE_PREC_MIXED}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libslse works on device tensors")


class Context:
    """An slse_ctx bound to one device (scratch memory, graphs, cached factor)."""

    def __init__(self, device=0):
        self.lib = L.load()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        L.check(self.lib.slse_ctx_create(ctypes.byref(h), self.device.index or 0))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.slse_ctx_destroy(self.h)
            self.h = None

    def trim(self):
        L.check(self.lib.slse_ctx_trim(self.h))

    def save_tuning(self, path):
        """slse_ctx_save_tuning: the tuned launch shapes to a text file."""
        L.check(self.lib.slse_ctx_save_tuning(self.h, str(path).encode()))

    def load_tuning(self, path):
        """slse_ctx_load_tuning: returns the number of entries taken (0 for a file
        written on another part)."""
        n = L.c_i32()
        L.check(self.lib.slse_ctx_load_tuning(self.h, str(path).encode(), ctypes.byref(n)))
        return n.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device=None):
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


def paper_params(d, r=None):
    """slse_paper_params: (r, mu, eta) with r = 6d unless given, eta = d/r and
    mu = (1 - eta)^2 (Sec. 5 parameter choice)."""
    lib = L.load()
    r_out, mu, eta = L.c_i64(), L.c_f64(), L.c_f64()
    L.check(lib.slse_paper_params(int(d), int(r or 0), ctypes.byref(r_out), ctypes.byref(mu),
                                  ctypes.byref(eta)))
    return r_out.value, mu.value, eta.value


def auto_a(m, d, omega=0.5, a1=None):
    """slse_stage1_counts: stage-1 counts from the lower bound of Thm
    lowerBoundai (Sec. 4); a_1 is `a1`, else a_2."""
    lib = L.load()
    K = len(m)
    marr = (L.c_i64 * K)(*[int(v) for v in m])
    out = (L.c_i32 * K)()
    L.check(lib.slse_stage1_counts(marr, K, int(d), float(omega), int(a1 or 0), out))
    return list(out)


def paper_schedule(n, d, m1_factor=8):
    """slse_paper_schedule: m_1 = 8d (rounded up to a power of 2), doubling to
    the largest power of 2 <= N/2 (Sec. 5)."""
    lib = L.load()
    cap = L.SLSE_MAX_LEVELS
    out = (L.c_i64 * cap)()
    K = L.c_i32()
    L.check(lib.slse_paper_schedule(int(n), int(d), int(m1_factor), out, cap, ctypes.byref(K)))
    return list(out[:K.value])


@dataclass
class Params:
    kind: str = "srht"
    seed: int = 0
    m: List[int] = field(default_factory=list)
    a: List[int] = field(default_factory=list)
    r: int = 0
    mu: Optional[float] = None
    eta: Optional[float] = None
    s_max: int = 20
    tol: float = 0.0
    precision: str = "f64"
    fp32_sweeps: int = 0
    momentum_reset: bool = False
    factor: str = "chol"
    use_graph: bool = False

    def to_c(self, d, beta0=None, trajectory=None, surrogate=None, beta_ref=None, rel_err=None,
             pred_err=None, start_step=0, stop_step=0, beta_prev=None, state_out=None):
        q = L.slse_params()
        q.kind = _KIND[self.kind]
        q.seed = self.seed
        q.K = len(self.m)
        if q.K > L.SLSE_MAX_LEVELS or len(self.a) != q.K:
            raise ValueError("m and a must have the same length <= SLSE_MAX_LEVELS")
        for i, (mi, ai) in enumerate(zip(self.m, self.a)):
            q.m[i] = int(mi)
            q.a[i] = int(ai)
        r, mu, eta = paper_params(d, self.r or None)
        q.r = r
        q.mu = mu if self.mu is None else self.mu
        q.eta = eta if self.eta is None else self.eta
        q.s_max = self.s_max
        q.tol = self.tol
        q.precision = _PREC[self.precision]
        q.fp32_sweeps = self.fp32_sweeps
        q.momentum_reset = 1 if self.momentum_reset else 0
        q.factor = _FACTOR[self.factor]
        q.beta0 = _ptr(beta0).value
        q.trajectory = _ptr(trajectory).value
        q.surrogate = _ptr(surrogate).value
        q.use_graph = 1 if self.use_graph else 0
        q.beta_ref = _ptr(beta_ref).value
        q.rel_err = _ptr(rel_err).value
        q.pred_err = _ptr(pred_err).value
        q.start_step = int(start_step)
        q.stop_step = int(stop_step)
        q.beta_prev = _ptr(beta_prev).value
        q.state_out = _ptr(state_out).value
        return q


def _problem(X, Y):
    _need_cuda(X, Y)
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D row-major")
    if Y.dim() != 1 or Y.stride(0) != 1 or Y.shape[0] != X.shape[0]:
        raise ValueError("Y must be contiguous with N entries")
    if X.dtype != Y.dtype or X.dtype not in _DT:
        raise ValueError("X and Y must share dtype float32 or float64")
    p = L.slse_problem()
    p.N, p.d = X.shape
    p.X = X.data_ptr()
    p.ldx = X.stride(0)
    p.Y = Y.data_ptr()
    p.dtype = _DT[X.dtype]
    return p


def _info(st, rep):
    return dict(status=L.STATUS_NAMES.get(st, st), stage1_steps=rep.stage1_steps,
                stage2_steps=rep.stage2_steps, surrogate0=rep.surrogate0,
                surrogate_final=rep.surrogate_final, ms_total=rep.ms_total,
                ms_sketch=rep.ms_sketch, ms_factor=rep.ms_factor, ms_stage1=rep.ms_stage1,
                ms_stage2=rep.ms_stage2)


def solve(X, Y, params: Params, ctx=None, beta0=None, record=False, report=True, beta_ref=None,
          pred_err=False, ws=None, start_step=0, stop_step=0, beta_prev=None, state_out=None):
    """slse_solve (slse_solve_ws when `ws`, a uint8 device tensor, is given).

    Returns (beta, report dict), plus (trajectory, surrogate) when `record`,
    plus the per-iterate errors against `beta_ref` as a dict with "rel_err"
    (and "pred_err" = ||X (beta_t - beta_ref)||^2 when `pred_err`) when
    `beta_ref` is given.  Checkpoint and resume: steps start_step ..
    stop_step - 1 (0 = to the end) are run from beta0 (beta_t) and beta_prev
    (beta_{t-1}); `state_out`, a (2, d) float64 device tensor, receives the
    state (beta_{t-1}, beta_t) after the last step run.
    """
    ctx = ctx or default_context(X.device.index)
    p = _problem(X, Y)
    d = X.shape[1]
    T = sum(params.a) + params.s_max
    traj = torch.empty((T + 1, d), dtype=torch.float64, device=X.device) if record else None
    sur = torch.empty(max(T, 1), dtype=torch.float64, device=X.device) if record else None
    errs = None
    if beta_ref is not None:
        _need_cuda(beta_ref)
        errs = {"rel_err": torch.empty(T + 1, dtype=torch.float64, device=X.device)}
        if pred_err:
            errs["pred_err"] = torch.empty(T + 1, dtype=torch.float64, device=X.device)
    for v in (beta_prev, state_out):
        if v is not None:
            _need_cuda(v)
    if state_out is not None and (state_out.dtype != torch.float64 or state_out.numel() < 2 * d
                                  or not state_out.is_contiguous()):
        raise ValueError("state_out must be a contiguous float64 tensor of 2 x d")
    q = params.to_c(d, beta0, traj, sur, beta_ref, errs and errs["rel_err"],
                    errs and errs.get("pred_err"), start_step, stop_step, beta_prev, state_out)
    beta = torch.empty(d, dtype=torch.float64, device=X.device)
    rep = L.slse_report()
    rp = ctypes.byref(rep) if report else None
    if ws is None:
        st = ctx.lib.slse_solve(ctx.h, ctypes.byref(p), ctypes.byref(q), _ptr(beta), rp,
                                _stream(X.device))
    else:
        _need_cuda(ws)
        st = ctx.lib.slse_solve_ws(ctx.h, ctypes.byref(p), ctypes.byref(q), _ptr(beta), rp,
                                   _ptr(ws), ws.numel() * ws.element_size(), _stream(X.device))
    if st not in (L.SLSE_OK, L.SLSE_ENOTCONV):
        L.check(st)
    out = (beta, _info(st, rep))
    if record:
        out = out + (traj, sur)
    if errs is not None:
        out = out + (errs,)
    return out


def workspace_size(X, Y, params: Params, ctx=None):
    """slse_workspace_size: device bytes slse_solve_ws needs for this solve."""
    ctx = ctx or default_context(X.device.index)
    p = _problem(X, Y)
    q = params.to_c(X.shape[1])
    n = ctypes.c_size_t()
    L.check(ctx.lib.slse_workspace_size(ctx.h, ctypes.byref(p), ctypes.byref(q), ctypes.byref(n)))
    return n.value


def ihs(X, Y, kind, seed, r, steps, ctx=None, beta0=None, record=False, factor="chol",
        precision=None, use_graph=False):
    """slse_ihs: IHS with a Hessian sketch drawn anew at each of `steps` full-data
    steps (key seed + t at step t).  Returns beta, or (beta, trajectory)."""
    ctx = ctx or default_context(X.device.index)
    p = _problem(X, Y)
    d = X.shape[1]
    prec = precision or ("mixed" if X.dtype == torch.float32 else "f64")
    prm = Params(kind=kind, seed=seed, m=[], a=[], r=r, s_max=steps, precision=prec, factor=factor,
                 use_graph=use_graph, mu=1.0, eta=0.0)
    traj = torch.empty((steps + 1, d), dtype=torch.float64, device=X.device) if record else None
    q = prm.to_c(d, beta0, traj)
    beta = torch.empty(d, dtype=torch.float64, device=X.device)
    L.check(ctx.lib.slse_ihs(ctx.h, ctypes.byref(p), ctypes.byref(q), _ptr(beta), None,
                             _stream(X.device)))
    return (beta, traj) if record else beta


def sketch_apply(X, Y, kind, seed, m, r, ctx=None, bf16=False):
    """slse_sketch_apply: returns (A, Ahat, layout dict).

    bf16=True asks for the Gaussian sketch of FP32 data on the matrix cores
    (BF16 operands, FP32 accumulation); A and Ahat are FP32.
    """
    ctx = ctx or default_context(X.device.index)
    p = _problem(X, Y)
    N, d = X.shape
    mK = list(m)
    rows_A = sum(mK) if kind == "countsketch" else mK[-1]
    es = X.element_size()
    align = 128 // es if d + 1 >= 128 // es else 16 // es  # rows of a full line start on a line
    ld = ((d + 1 + align - 1) // align) * align
    A = torch.empty((rows_A, ld), dtype=X.dtype, device=X.device)
    Ah = torch.empty((r, ld), dtype=X.dtype, device=X.device)
    marr = (ctypes.c_int64 * len(mK))(*mK)
    lay = L.slse_sketch_layout()
    out_t = L.SLSE_BF16 if bf16 else p.dtype
    L.check(ctx.lib.slse_sketch_apply(ctx.h, _KIND[kind], seed, N, d, _ptr(X), p.ldx, _ptr(Y),
                                      p.dtype, marr, len(mK), r, _ptr(A), ld, _ptr(Ah), ld,
                                      out_t, ctypes.byref(lay), _stream(X.device)))
    layout = dict(K=lay.K, m=list(lay.m[:lay.K]), offset=list(lay.offset[:lay.K]),
                  scale=list(lay.scale[:lay.K]), rows_A=lay.rows_A, r=lay.r,
                  hat_scale=lay.hat_scale, n_pad=lay.n_pad)
    return A[:, : d + 1], Ah[:, : d + 1], layout


def factor(A, d, scale, method="chol", ctx=None):
    """slse_factor on the first d columns of A: returns (R, M)."""
    ctx = ctx or default_context(A.device.index)
    _need_cuda(A)
    if A.stride(1) != 1 or A.dtype not in _DT:
        raise ValueError("A must be row-major float32/float64")
    R = torch.empty((d, d), dtype=torch.float64, device=A.device)
    M = torch.empty((d, d), dtype=torch.float64, device=A.device)
    L.check(ctx.lib.slse_factor(ctx.h, A.shape[0], d, _ptr(A), A.stride(0), _DT[A.dtype], scale,
                                _FACTOR[method], _ptr(R), d, _ptr(M), d, _stream(A.device)))
    return R, M


def fused_resid_grad(X, Y, beta, scale=1.0, accum="f64", ctx=None, n=None):
    """slse_fused_resid_grad: g = scale X^T (Y - X beta) and scale ||Y - X beta||^2."""
    ctx = ctx or default_context(X.device.index)
    _need_cuda(X, beta)
    if X.stride(1) != 1 or X.dtype not in _DT:
        raise ValueError("X must be row-major float32/float64")
    if Y is not None and (Y.stride(0) != 1 or Y.dtype != X.dtype):
        raise ValueError("Y must be contiguous with X's dtype")
    n = X.shape[0] if n is None else n
    d = X.shape[1]
    g = torch.empty(d, dtype=torch.float64, device=X.device)
    rn = torch.empty(1, dtype=torch.float64, device=X.device)
    L.check(ctx.lib.slse_fused_resid_grad(ctx.h, n, d, _ptr(X), X.stride(0), _ptr(Y), _DT[X.dtype],
                                          _ptr(beta), scale, _DT[torch.float64 if accum == "f64" else torch.float32],
                                          _ptr(g), _ptr(rn), _stream(X.device)))
    return g, rn


def fused_resid_grad_noalloc(X, Y, beta, scale=1.0, accum="f64", ctx=None, n=None, g=None, rn=None):
    """slse_fused_resid_grad_noalloc: the same pass with the library's fixed
    scratch (no device allocation inside the call; g and rn may be passed in)."""
    ctx = ctx or default_context(X.device.index)
    _need_cuda(X, beta)
    if X.stride(1) != 1 or X.dtype not in _DT:
        raise ValueError("X must be row-major float32/float64")
    if Y is not None and (Y.stride(0) != 1 or Y.dtype != X.dtype):
        raise ValueError("Y must be contiguous with X's dtype")
    n = X.shape[0] if n is None else n
    d = X.shape[1]
    g = torch.empty(d, dtype=torch.float64, device=X.device) if g is None else g
    rn = torch.empty(1, dtype=torch.float64, device=X.device) if rn is None else rn
    L.check(ctx.lib.slse_fused_resid_grad_noalloc(
        ctx.h, n, d, _ptr(X), X.stride(0), _ptr(Y), _DT[X.dtype], _ptr(beta), scale,
        _DT[torch.float64 if accum == "f64" else torch.float32], _ptr(g), _ptr(rn),
        _stream(X.device)))
    return g, rn


def backward(X, Y, params: Params, beta_hat, w, grad_dtype=None, ctx=None, want_dX=True, want_dY=True):
    """slse_backward: returns (dX, dY, lambda).  w is a float64 device vector of
    any stride (read in place)."""
    ctx = ctx or default_context(X.device.index)
    p = _problem(X, Y)
    _need_cuda(w, beta_hat)
    if w.dtype != torch.float64 or w.dim() != 1 or w.shape[0] != X.shape[1]:
        raise ValueError("w must be a float64 vector of length d")
    N, d = X.shape
    gd = X.dtype if grad_dtype is None else grad_dtype
    dX = torch.empty((N, d), dtype=gd, device=X.device) if want_dX else None
    dY = torch.empty(N, dtype=gd, device=X.device) if want_dY else None
    lam = torch.empty(d, dtype=torch.float64, device=X.device)
    q = params.to_c(d)
    rep = L.slse_report()
    L.check(ctx.lib.slse_backward(ctx.h, ctypes.byref(p), ctypes.byref(q), _ptr(beta_hat), _ptr(w),
                                  w.stride(0), _ptr(dX), d, _ptr(dY), _DT[gd], _ptr(lam),
                                  ctypes.byref(rep), _stream(X.device)))
    return dX, dY, lam


def debug_stream(what, seed, stream_id, aux, start, count, device=0, ctx=None):
    ctx = ctx or default_context(device)
    n = 4 * count if what == 0 else count
    out = torch.empty(max(n, 1), dtype=torch.int64, device=torch.device("cuda", device))
    L.check(ctx.lib.slse_debug_stream(ctx.h, what, seed, stream_id, aux, start, count, _ptr(out),
                                      _stream(device)))
    return out[:n]


def debug_batch_plan(shapes, params_list, dtype=torch.float32):
    """slse_debug_batch_plan on problems of the given (N, d) shapes (host only:
    no tensors, fake 256-byte aligned data pointers).  Returns the device bytes
    the batch needs, or raises the plan check's error."""
    B = len(shapes)
    probs = (L.slse_problem * B)()
    qs = (L.slse_params * B)()
    for b, (n, d) in enumerate(shapes):
        probs[b].N, probs[b].d = n, d
        probs[b].X = (1 << 44) + b * (1 << 36)
        probs[b].ldx = d
        probs[b].Y = (1 << 44) + b * (1 << 36) + (1 << 35)
        probs[b].dtype = _DT[dtype]
        qs[b] = params_list[b].to_c(d)
    n = ctypes.c_size_t()
    L.check(L.load().slse_debug_batch_plan(B, probs, qs, ctypes.byref(n)))
    return n.value


def debug_gaussian(seed, stream_id, k0, nk, j0, nj, device=0, ctx=None, form=0):
    ctx = ctx or default_context(device)
    out = torch.empty((max(nk, 1), max(nj, 1)), dtype=torch.float64, device=torch.device("cuda", device))
    L.check(ctx.lib.slse_debug_gaussian(ctx.h, seed, stream_id, form, k0, nk, j0, nj, _ptr(out),
                                        _stream(device)))
    return out[:nk, :nj]


def debug_bandwidth(mode, src, dst, nbytes=None, blocks=0, ctx=None):
    """slse_debug_bandwidth: a plain streaming read (mode 0, one word per block
    into dst) or copy (mode 1) of a device tensor's bytes."""
    ctx = ctx or default_context(src.device.index)
    _need_cuda(src, dst)
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    L.check(ctx.lib.slse_debug_bandwidth(ctx.h, mode, _ptr(src), _ptr(dst), nbytes - nbytes % 16,
                                         blocks, _stream(src.device)))


def debug_gaussian_generate(seed, stream_id, m, N, blocks=1024, device=0, ctx=None, sink=None):
    """slse_debug_gaussian_generate: generate the m x N entries of G alone."""
    ctx = ctx or default_context(device)
    sink = torch.empty(256 * blocks, dtype=torch.int32, device=torch.device("cuda", device)) \
        if sink is None else sink
    L.check(ctx.lib.slse_debug_gaussian_generate(ctx.h, seed, stream_id, int(m), int(N), blocks,
                                                 _ptr(sink), _stream(device)))
    return sink


def debug_gaussian_plan(N, d, m, bf16):
    """Data-row splits of a Gaussian sketch (host only)."""
    s = L.c_i32()
    L.check(L.load().slse_debug_gaussian_plan(int(N), int(d), int(m), 1 if bf16 else 0,
                                              ctypes.byref(s)))
    return s.value


class SLSEFunction(torch.autograd.Function):
    """beta_hat = SLSE-FRS(X, Y) with the hand-written adjoint of slse_backward."""

    @staticmethod
    def forward(ctx, X, Y, params):
        beta, _ = solve(X, Y, params)
        ctx.save_for_backward(X, Y, beta)
        ctx.params = params
        return beta

    @staticmethod
    def backward(ctx, w):
        # w has beta's dtype (float64); any stride is read in place by the library
        X, Y, beta = ctx.saved_tensors
        dX, dY, _ = backward(X, Y, ctx.params, beta, w, want_dX=ctx.needs_input_grad[0],
                             want_dY=ctx.needs_input_grad[1])
        return dX, dY, None


def solve_batched(Xs, Ys, params_list, ctx=None, report=True):
    """slse_solve_batched: returns (list of betas, list of report dicts)."""
    B = len(Xs)
    if not (len(Ys) == B == len(params_list)):
        raise ValueError("Xs, Ys and params_list must have the same length")
    if B == 0:
        return [], []
    ctx = ctx or default_context(Xs[0].device.index)
    probs = (L.slse_problem * B)()
    qs = (L.slse_params * B)()
    betas = []
    for b in range(B):
        probs[b] = _problem(Xs[b], Ys[b])
        qs[b] = params_list[b].to_c(Xs[b].shape[1])
        betas.append(torch.empty(Xs[b].shape[1], dtype=torch.float64, device=Xs[b].device))
    ptrs = (ctypes.c_void_p * B)(*[b.data_ptr() for b in betas])
    reps = (L.slse_report * B)()
    st = ctx.lib.slse_solve_batched(ctx.h, B, probs, qs, ptrs, reps if report else None,
                                    _stream(Xs[0].device))
    if st not in (L.SLSE_OK, L.SLSE_ENOTCONV):
        L.check(st)
    infos = [dict(status=L.STATUS_NAMES.get(r.status, r.status), stage1_steps=r.stage1_steps,
                  stage2_steps=r.stage2_steps) for r in reps] if report else []
    return betas, infos
