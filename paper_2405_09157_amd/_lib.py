"""ctypes binding of the C ABI in include/scp_mwu.h (argument marshalling only).

Every computation happens in ``libscpmwu.so`` (HIP kernels for gfx950 and
their host driver).  Importing this module fails loudly when the library has
not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libscpmwu.so")

# ---- constants (mirror include/scp_mwu.h)
SCP_MWU_ABI_VERSION = 1
SCP_MWU_PROBLEM_SES, SCP_MWU_PROBLEM_SVM = 1, 2
SCP_MWU_F32, SCP_MWU_BF16, SCP_MWU_F64, SCP_MWU_FP8 = 1, 2, 3, 4
SCP_MWU_OK, SCP_MWU_STOPPED = 0, 1
SCP_MWU_E_INVAL, SCP_MWU_E_NOMEM, SCP_MWU_E_HIP, SCP_MWU_E_STATE = -1, -2, -3, -4
SCP_MWU_E_NUMERIC, SCP_MWU_E_INFEASIBLE, SCP_MWU_E_UNSUPPORTED = -5, -6, -7
SCP_MWU_OUT_RUNNING, SCP_MWU_OUT_SEPARATED, SCP_MWU_OUT_BEAT = 0, 1, 2
SCP_MWU_OUT_STABILIZED, SCP_MWU_OUT_T_REACHED, SCP_MWU_OUT_NUMERIC = 3, 4, 5
SCP_MWU_FLAG_NO_EARLY_STOP, SCP_MWU_FLAG_THEORY, SCP_MWU_FLAG_CERTIFICATES = 1, 2, 4
SCP_MWU_FLAG_DETERMINISTIC = 8

OUTCOME_NAMES = {0: "running", 1: "separated", 2: "beat_alpha", 3: "stabilized",
                 4: "t_reached", 5: "numeric"}

# symbols the header declares (checked by the CPU test suite)
EXPORTS = ("scp_mwu_init", "scp_mwu_step", "scp_mwu_solve", "scp_mwu_backward", "scp_mwu_backward_noalloc",
           "scp_mwu_product_init",
           "scp_mwu_product_exp", "scp_mwu_product_destroy",
           "scp_mwu_get_state", "scp_mwu_set_state", "scp_mwu_get_vector", "scp_mwu_get_D",
           "scp_mwu_destroy", "scp_mwu_last_error", "scp_mwu_strerror", "scp_mwu_cast_bf16",
           "scp_mwu_time_passes", "scp_mwu_read_reference", "scp_mwu_quantize_fp8",
           "scp_mwu_batch_init", "scp_mwu_batch_step", "scp_mwu_batch_solve", "scp_mwu_batch_get_vector",
           "scp_mwu_batch_get_D", "scp_mwu_batch_time_iters", "scp_mwu_batch_destroy",
           "scp_mwu_batch_last_error", "scp_mwu_batch_solve_kway")


class scp_mwu_desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("problem", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int64),
        ("ld", ctypes.c_int64),
        ("points", ctypes.c_void_p),
        ("radii", ctypes.c_void_p),
        ("n_pos", ctypes.c_int64),
        ("v1_index", ctypes.c_int64),
        ("eps", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("patience", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("t_cap", ctypes.c_int64),
        ("max_iters", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("chunk", ctypes.c_int32),
        ("grid", ctypes.c_int32),
    ]


class scp_mwu_stepinfo(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int64),
        ("t_end", ctypes.c_int64),
        ("T", ctypes.c_int64),
        ("outcome", ctypes.c_int32),
        ("degenerate", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("f_last", ctypes.c_double),
        ("f_best", ctypes.c_double),
        ("t_best", ctypes.c_int64),
        ("value", ctypes.c_double),
        ("scale", ctypes.c_double),
        ("log_trace", ctypes.c_double),
        ("bound", ctypes.c_double),
    ]


class scp_mwu_result(ctypes.Structure):
    _fields_ = [
        ("value", ctypes.c_double),
        ("lower", ctypes.c_double),
        ("upper", ctypes.c_double),
        ("search_lo", ctypes.c_double),
        ("search_hi", ctypes.c_double),
        ("D", ctypes.c_double),
        ("iters", ctypes.c_int64),
        ("tests", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("passes", ctypes.c_int64),
    ]


class scp_mwu_batch_desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("dtype", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("count", ctypes.c_int32),
        ("n", ctypes.POINTER(ctypes.c_int64)),
        ("d", ctypes.POINTER(ctypes.c_int64)),
        ("offset", ctypes.POINTER(ctypes.c_int64)),
        ("points", ctypes.c_void_p),
        ("eps", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("patience", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("t_cap", ctypes.c_int64),
        ("max_iters", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("chunk", ctypes.c_int32),
        ("rows_per_group", ctypes.c_int32),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libscpmwu.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2405_09157_amd.build` (no fallback path exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "scp_mwu_init": (i32, [P(scp_mwu_desc), P(vp)]),
        "scp_mwu_step": (i32, [vp, f64, i64, i32, i32, P(scp_mwu_stepinfo)]),
        "scp_mwu_solve": (i32, [vp, P(scp_mwu_result), P(f64)]),
        "scp_mwu_backward": (i32, [vp, f64, P(ctypes.c_float), P(f64), i32]),
        "scp_mwu_backward_noalloc": (i32, [vp, f64, P(ctypes.c_float), P(f64), i32]),
        "scp_mwu_product_init": (i32, [i64, P(i64), i64, i64, vp, P(vp)]),
        "scp_mwu_product_exp": (i32, [vp, vp, f64, vp, P(f64)]),
        "scp_mwu_product_destroy": (None, [vp]),
        "scp_mwu_get_state": (i32, [vp, P(f64), P(i64)]),
        "scp_mwu_set_state": (i32, [vp, f64, i64, i64, P(f64)]),
        "scp_mwu_get_vector": (i32, [vp, i32, P(f64)]),
        "scp_mwu_get_D": (i32, [vp, P(f64)]),
        "scp_mwu_destroy": (None, [vp]),
        "scp_mwu_last_error": (ctypes.c_char_p, [vp]),
        "scp_mwu_strerror": (ctypes.c_char_p, [i32]),
        "scp_mwu_cast_bf16": (i32, [vp, vp, i64, vp]),
        "scp_mwu_time_passes": (i32, [vp, i32, P(f64), P(f64)]),
        "scp_mwu_read_reference": (i32, [vp, i64, i32, vp, P(f64)]),
        "scp_mwu_quantize_fp8": (i32, [vp, i64, i64, i64, vp, vp, vp]),
        "scp_mwu_batch_init": (i32, [P(scp_mwu_batch_desc), P(vp)]),
        "scp_mwu_batch_step": (i32, [vp, P(f64), P(i64), i32, i32, P(scp_mwu_stepinfo)]),
        "scp_mwu_batch_solve": (i32, [vp, P(scp_mwu_result), P(f64)]),
        "scp_mwu_batch_solve_kway": (i32, [vp, P(scp_mwu_result), P(f64)]),
        "scp_mwu_batch_get_vector": (i32, [vp, i32, P(f64)]),
        "scp_mwu_batch_get_D": (i32, [vp, P(f64)]),
        "scp_mwu_batch_time_iters": (i32, [vp, i32, P(f64), P(f64)]),
        "scp_mwu_batch_destroy": (None, [vp]),
        "scp_mwu_batch_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ScpMwuError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


def _check(code: int, ctx=None) -> int:
    if code < 0:
        lib = load()
        text = lib.scp_mwu_last_error(ctx).decode() or lib.scp_mwu_strerror(code).decode()
        raise ScpMwuError(code, text)
    return code


# ---- thin wrappers with the C names
def scp_mwu_init(desc: scp_mwu_desc) -> ctypes.c_void_p:
    lib = load()
    ctx = ctypes.c_void_p()
    _check(lib.scp_mwu_init(ctypes.byref(desc), ctypes.byref(ctx)))
    return ctx


def scp_mwu_step(ctx, alpha: float, T: int, k: int, reset: int = 0) -> scp_mwu_stepinfo:
    info = scp_mwu_stepinfo()
    _check(load().scp_mwu_step(ctx, alpha, T, k, reset, ctypes.byref(info)), ctx)
    return info


def scp_mwu_solve(ctx, d: int):
    res = scp_mwu_result()
    y = (ctypes.c_double * (d + 2))()
    code = _check(load().scp_mwu_solve(ctx, ctypes.byref(res), y), ctx)
    return code, res, list(y)


def scp_mwu_backward(ctx, grad_value: float, grad_points_ptr, checkpoint_every: int = 50) -> float:
    """grad_value * dR/dV into the device buffer at grad_points_ptr (None: the
    forward map only); returns R."""
    value = ctypes.c_double()
    gp = ctypes.cast(grad_points_ptr, ctypes.POINTER(ctypes.c_float)) if grad_points_ptr else None
    _check(load().scp_mwu_backward(ctx, grad_value, gp, ctypes.byref(value), int(checkpoint_every)), ctx)
    return value.value


def scp_mwu_backward_noalloc(ctx, grad_value: float, grad_points_ptr, checkpoint_every: int = 50) -> float:
    """scp_mwu_backward on the library's static workspace (no allocation)."""
    value = ctypes.c_double()
    gp = ctypes.cast(grad_points_ptr, ctypes.POINTER(ctypes.c_float)) if grad_points_ptr else None
    _check(load().scp_mwu_backward_noalloc(ctx, grad_value, gp, ctypes.byref(value), int(checkpoint_every)), ctx)
    return value.value


def scp_mwu_product_init(n_orth: int, offsets, length: int, stream: int = 0) -> ctypes.c_void_p:
    """Handle of the product-cone layout R^{n_orth}_+ (+) Lorentz blocks at
    `offsets` (a sequence or an int64 numpy array of nblocks + 1 values, empty
    without blocks) over vectors of `length` values."""
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int64) if len(offsets) else None
    k = max(len(offsets) - 1, 0)
    ptr = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if off is not None else None
    h = ctypes.c_void_p()
    code = load().scp_mwu_product_init(int(n_orth), ptr, k, int(length), stream, ctypes.byref(h))
    if code != SCP_MWU_OK:
        raise ScpMwuError(code, "scp_mwu_product_init: " + load().scp_mwu_strerror(code).decode())
    return h


def scp_mwu_product_exp(handle, m_ptr: int, eta: float, p_ptr: int, want_log_trace: bool = True):
    """p = exp(-eta m) / Tr(...) on the handle's layout; returns ln Tr (waiting
    for the stream) or None (launches only enqueued)."""
    lt = ctypes.c_double()
    code = load().scp_mwu_product_exp(handle, m_ptr, float(eta), p_ptr, ctypes.byref(lt) if want_log_trace else None)
    if code != SCP_MWU_OK:
        raise ScpMwuError(code, "scp_mwu_product_exp: " + load().scp_mwu_strerror(code).decode())
    return lt.value if want_log_trace else None


def scp_mwu_product_destroy(handle) -> None:
    load().scp_mwu_product_destroy(handle)


def scp_mwu_get_state(ctx, d: int, svm: bool):
    buf = (ctypes.c_double * (d + 2))()
    t = ctypes.c_int64()
    _check(load().scp_mwu_get_state(ctx, buf, ctypes.byref(t)), ctx)
    return list(buf)[: d + (2 if svm else 0)], t.value


def scp_mwu_set_state(ctx, alpha: float, T: int, t: int, sums) -> None:
    arr = (ctypes.c_double * len(sums))(*[float(v) for v in sums])
    _check(load().scp_mwu_set_state(ctx, alpha, T, t, arr), ctx)


def scp_mwu_get_vector(ctx, which: int, d: int, svm: bool):
    buf = (ctypes.c_double * (d + 2))()
    _check(load().scp_mwu_get_vector(ctx, which, buf), ctx)
    return list(buf)[: d + (2 if svm else 0)]


def scp_mwu_get_D(ctx) -> float:
    D = ctypes.c_double()
    _check(load().scp_mwu_get_D(ctx, ctypes.byref(D)), ctx)
    return D.value


def scp_mwu_destroy(ctx) -> None:
    load().scp_mwu_destroy(ctx)


def scp_mwu_cast_bf16(src_ptr: int, dst_ptr: int, n: int, stream: int = 0) -> None:
    _check(load().scp_mwu_cast_bf16(src_ptr, dst_ptr, n, stream))


def scp_mwu_time_passes(ctx, k: int):
    """(mean streaming-pass kernel ms, mean whole-iteration ms) over k iterations."""
    mp, mi = ctypes.c_double(), ctypes.c_double()
    _check(load().scp_mwu_time_passes(ctx, k, ctypes.byref(mp), ctypes.byref(mi)), ctx)
    return mp.value, mi.value


def scp_mwu_quantize_fp8(src_ptr: int, n: int, d: int, ld: int, codes_ptr: int, scales_ptr: int,
                         stream: int = 0) -> None:
    _check(load().scp_mwu_quantize_fp8(src_ptr, n, d, ld, codes_ptr, scales_ptr, stream))


def scp_mwu_read_reference(ptr: int, nbytes: int, reps: int = 20, stream: int = 0) -> float:
    """Mean ms of a plain streaming read of nbytes at device address ptr."""
    ms = ctypes.c_double()
    _check(load().scp_mwu_read_reference(ptr, nbytes, reps, stream, ctypes.byref(ms)))
    return ms.value


def scp_mwu_strerror(code: int) -> str:
    return load().scp_mwu_strerror(code).decode()


# ---- batched SES
def _check_batch(code: int, b=None) -> int:
    if code < 0:
        lib = load()
        text = lib.scp_mwu_batch_last_error(b).decode() or lib.scp_mwu_strerror(code).decode()
        raise ScpMwuError(code, text)
    return code


def scp_mwu_batch_init(desc: scp_mwu_batch_desc) -> ctypes.c_void_p:
    b = ctypes.c_void_p()
    _check_batch(load().scp_mwu_batch_init(ctypes.byref(desc), ctypes.byref(b)))
    return b


def scp_mwu_batch_step(b, alpha, T, k: int, reset: int = 0):
    m = len(alpha)
    a = (ctypes.c_double * m)(*[float(v) for v in alpha])
    t = (ctypes.c_int64 * m)(*[int(v) for v in T])
    info = (scp_mwu_stepinfo * m)()
    _check_batch(load().scp_mwu_batch_step(b, a, t, k, reset, info), b)
    return list(info)


def scp_mwu_batch_solve(b, m: int, d_total: int):
    res = (scp_mwu_result * m)()
    y = (ctypes.c_double * (d_total + m))()
    code = _check_batch(load().scp_mwu_batch_solve(b, res, y), b)
    return code, list(res), list(y)


def scp_mwu_batch_solve_kway(b, d: int):
    res = scp_mwu_result()
    y = (ctypes.c_double * (d + 1))()
    code = _check_batch(load().scp_mwu_batch_solve_kway(b, ctypes.byref(res), y), b)
    return code, res, list(y)


def scp_mwu_batch_get_vector(b, which: int, d_total: int):
    y = (ctypes.c_double * d_total)()
    _check_batch(load().scp_mwu_batch_get_vector(b, which, y), b)
    return list(y)


def scp_mwu_batch_get_D(b, m: int):
    D = (ctypes.c_double * m)()
    _check_batch(load().scp_mwu_batch_get_D(b, D), b)
    return list(D)


def scp_mwu_batch_time_iters(b, k: int):
    mp, mi = ctypes.c_double(), ctypes.c_double()
    _check_batch(load().scp_mwu_batch_time_iters(b, k, ctypes.byref(mp), ctypes.byref(mi)), b)
    return mp.value, mi.value


def scp_mwu_batch_destroy(b) -> None:
    load().scp_mwu_batch_destroy(b)
