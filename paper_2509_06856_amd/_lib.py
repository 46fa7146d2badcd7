"""ctypes binding of libslse (argument marshalling only).

Every entry point of include/slse.h is exposed under the same name.  Device
memory and streams come from PyTorch tensors (`tensor.data_ptr()`,
`torch.cuda.current_stream().cuda_stream`); every step of the path runs in the
library's HIP kernels.  Loading fails loudly when the library is missing.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SLSE_LIB", os.path.join(HERE, "libslse.so"))

SLSE_MAX_LEVELS = 40

# enums
SLSE_OK = 0
SLSE_EINVAL = -1
SLSE_ENOMEM = -2
SLSE_EDEVICE = -3
SLSE_ESINGULAR = -4
SLSE_ENOTCONV = -5
SLSE_ENONFINITE = -6
SLSE_EUNSUPPORTED = -7
STATUS_NAMES = {
    0: "SLSE_OK", -1: "SLSE_EINVAL", -2: "SLSE_ENOMEM", -3: "SLSE_EDEVICE",
    -4: "SLSE_ESINGULAR", -5: "SLSE_ENOTCONV", -6: "SLSE_ENONFINITE", -7: "SLSE_EUNSUPPORTED",
}

SLSE_F32, SLSE_F64, SLSE_BF16 = 0, 1, 2
SLSE_SRHT, SLSE_COUNTSKETCH, SLSE_GAUSSIAN = 0, 1, 2
SLSE_FACTOR_CHOL, SLSE_FACTOR_QR = 0, 1
SLSE_PREC_F64, SLSE_PREC_MIXED = 0, 1

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_u64 = ctypes.c_uint64
c_f64 = ctypes.c_double
c_vp = ctypes.c_void_p


class slse_sketch_layout(ctypes.Structure):
    _fields_ = [
        ("K", c_i32),
        ("m", c_i64 * SLSE_MAX_LEVELS),
        ("offset", c_i64 * SLSE_MAX_LEVELS),
        ("scale", c_f64 * SLSE_MAX_LEVELS),
        ("rows_A", c_i64),
        ("r", c_i64),
        ("hat_scale", c_f64),
        ("n_pad", c_i64),
    ]


class slse_problem(ctypes.Structure):
    _fields_ = [
        ("N", c_i64),
        ("d", c_i64),
        ("X", c_vp),
        ("ldx", c_i64),
        ("Y", c_vp),
        ("dtype", c_i32),
    ]


class slse_params(ctypes.Structure):
    _fields_ = [
        ("kind", c_i32),
        ("seed", c_u64),
        ("K", c_i32),
        ("m", c_i64 * SLSE_MAX_LEVELS),
        ("a", c_i32 * SLSE_MAX_LEVELS),
        ("r", c_i64),
        ("mu", c_f64),
        ("eta", c_f64),
        ("s_max", c_i32),
        ("tol", c_f64),
        ("precision", c_i32),
        ("fp32_sweeps", c_i32),
        ("momentum_reset", c_i32),
        ("factor", c_i32),
        ("beta0", c_vp),
        ("trajectory", c_vp),
        ("surrogate", c_vp),
        ("use_graph", c_i32),
        ("beta_ref", c_vp),
        ("rel_err", c_vp),
        ("pred_err", c_vp),
        ("start_step", c_i32),
        ("stop_step", c_i32),
        ("beta_prev", c_vp),
        ("state_out", c_vp),
    ]


class slse_report(ctypes.Structure):
    _fields_ = [
        ("status", c_i32),
        ("stage1_steps", c_i32),
        ("stage2_steps", c_i32),
        ("surrogate0", c_f64),
        ("surrogate_final", c_f64),
        ("ms_total", c_f64),
        ("ms_sketch", c_f64),
        ("ms_factor", c_f64),
        ("ms_stage1", c_f64),
        ("ms_stage2", c_f64),
    ]


SIGNATURES = {
    "slse_last_error": (ctypes.c_char_p, []),
    "slse_version": (ctypes.c_char_p, []),
    "slse_ctx_create": (c_i32, [ctypes.POINTER(c_vp), c_i32]),
    "slse_ctx_destroy": (c_i32, [c_vp]),
    "slse_ctx_trim": (c_i32, [c_vp]),
    "slse_ctx_save_tuning": (c_i32, [c_vp, ctypes.c_char_p]),
    "slse_ctx_load_tuning": (c_i32, [c_vp, ctypes.c_char_p, ctypes.POINTER(c_i32)]),
    "slse_sketch_apply": (c_i32, [c_vp, c_i32, c_u64, c_i64, c_i64, c_vp, c_i64, c_vp, c_i32,
                                  ctypes.POINTER(c_i64), c_i32, c_i64, c_vp, c_i64, c_vp, c_i64,
                                  c_i32, ctypes.POINTER(slse_sketch_layout), c_vp]),
    "slse_factor": (c_i32, [c_vp, c_i64, c_i64, c_vp, c_i64, c_i32, c_f64, c_i32, c_vp, c_i64,
                            c_vp, c_i64, c_vp]),
    "slse_fused_resid_grad": (c_i32, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_i32, c_vp, c_f64,
                                      c_i32, c_vp, c_vp, c_vp]),
    "slse_fused_resid_grad_noalloc": (c_i32, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_i32, c_vp,
                                              c_f64, c_i32, c_vp, c_vp, c_vp]),
    "slse_solve": (c_i32, [c_vp, ctypes.POINTER(slse_problem), ctypes.POINTER(slse_params), c_vp,
                           ctypes.POINTER(slse_report), c_vp]),
    "slse_workspace_size": (c_i32, [c_vp, ctypes.POINTER(slse_problem), ctypes.POINTER(slse_params),
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "slse_solve_ws": (c_i32, [c_vp, ctypes.POINTER(slse_problem), ctypes.POINTER(slse_params), c_vp,
                              ctypes.POINTER(slse_report), c_vp, ctypes.c_size_t, c_vp]),
    "slse_ihs": (c_i32, [c_vp, ctypes.POINTER(slse_problem), ctypes.POINTER(slse_params), c_vp,
                         ctypes.POINTER(slse_report), c_vp]),
    "slse_paper_schedule": (c_i32, [c_i64, c_i64, c_i64, ctypes.POINTER(c_i64), c_i32,
                                    ctypes.POINTER(c_i32)]),
    "slse_paper_params": (c_i32, [c_i64, c_i64, ctypes.POINTER(c_i64), ctypes.POINTER(c_f64),
                                  ctypes.POINTER(c_f64)]),
    "slse_stage1_counts": (c_i32, [ctypes.POINTER(c_i64), c_i32, c_i64, c_f64, c_i32,
                                   ctypes.POINTER(c_i32)]),
    "slse_backward": (c_i32, [c_vp, ctypes.POINTER(slse_problem), ctypes.POINTER(slse_params),
                              c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i32, c_vp,
                              ctypes.POINTER(slse_report), c_vp]),
    "slse_solve_batched": (c_i32, [c_vp, c_i32, ctypes.POINTER(slse_problem),
                                   ctypes.POINTER(slse_params), ctypes.POINTER(c_vp),
                                   ctypes.POINTER(slse_report), c_vp]),
    "slse_debug_stream": (c_i32, [c_vp, c_i32, c_u64, c_i32, c_i64, c_i64, c_i64, c_vp, c_vp]),
    "slse_debug_gaussian": (c_i32, [c_vp, c_u64, c_i32, c_i32, c_i64, c_i64, c_i64, c_i64, c_vp,
                                    c_vp]),
    "slse_debug_gaussian_generate": (c_i32, [c_vp, c_u64, c_i32, c_i64, c_i64, c_i32, c_vp, c_vp]),
    "slse_debug_gaussian_plan": (c_i32, [c_i64, c_i64, c_i64, c_i32, ctypes.POINTER(c_i32)]),
    "slse_debug_batch_tiles": (c_i32, [c_i32, c_vp, c_vp, c_vp, c_i64, c_i64, c_vp, c_vp]),
    "slse_debug_bandwidth": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_i64, c_i32, c_vp]),
    "slse_debug_batch_plan": (c_i32, [c_i32, ctypes.POINTER(slse_problem), ctypes.POINTER(slse_params),
                                      ctypes.POINTER(ctypes.c_size_t)]),
}

_lib = None


def load(path=None):
    """Load libslse.so (raises if it is missing)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"libslse.so not found at {p}: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
        )
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SlseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status != SLSE_OK:
        msg = load().slse_last_error().decode(errors="replace")
        raise SlseError(status, msg)
    return status
