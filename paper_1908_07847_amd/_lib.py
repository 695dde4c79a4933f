"""ctypes binding of libmlp.so (the C ABI declared in include/mlp.h).

Argument marshalling only: every step of training runs in the HIP kernels
of the library.  If the library is missing this module raises at import
time -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# MLP_LIBRARY names another build of the same library (the host-sanitizer
# build the ABI tests run against); default: the in-tree libmlp.so.
LIB_PATH = os.environ.get("MLP_LIBRARY") or os.path.join(_PKG, "libmlp.so")

(MLP_OK, MLP_ERR_ARG, MLP_ERR_SHAPE, MLP_ERR_ALIGN, MLP_ERR_WORKSPACE, MLP_ERR_UNSUPPORTED, MLP_ERR_HIP,
 MLP_ERR_TIMEOUT, MLP_ERR_NONFINITE) = range(9)
PREC = {"fp32": 0, "bf16": 1, "e4m3": 2}
MLP_F_COMPENSATED = 1
SMALL_MAX_ROWS, SMALL_MAX_HIDDEN, SMALL_MAX_IN, SMALL_MAX_OUT = 128, 64, 48, 4
MAX_SHARED_NETS = 64
STATIC_SCRATCH_BYTES = 32 << 20   # MLP_STATIC_SCRATCH_BYTES


class MLPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libmlp status {status}: {message}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("n_rows", ctypes.c_int64), ("batch", ctypes.c_int64),
                ("lr", ctypes.c_float), ("flags", ctypes.c_uint32)]


class Params(ctypes.Structure):
    _fields_ = [("W1", ctypes.c_void_p), ("b1", ctypes.c_void_p), ("W2", ctypes.c_void_p),
                ("b2", ctypes.c_void_p)]


class BatchItem(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("lr", ctypes.c_float),
                ("reserved", ctypes.c_int32), ("x_off", ctypes.c_int64), ("p_off", ctypes.c_int64)]


class LaunchHint(ctypes.Structure):
    _fields_ = [("small_threads", ctypes.c_int32), ("large_row_blocks", ctypes.c_int32),
                ("large_hidden_blocks", ctypes.c_int32), ("large_waves", ctypes.c_int32)]


assert ctypes.sizeof(BatchItem) == 32 and ctypes.sizeof(Config) == 40 and ctypes.sizeof(LaunchHint) == 16

# Every symbol include/mlp.h declares.
F_COMPENSATED, F_DETERMINISTIC, F_CHECK_FINITE, F_TANH_HIDDEN = 1, 2, 4, 8   # mlp_config flags
BARRIER_PROBE_WS_BYTES = 2048   # MLP_BARRIER_PROBE_WS_BYTES

SYMBOLS = ["mlp_workspace_size", "mlp_init", "mlp_destroy", "mlp_forward", "mlp_backward", "mlp_step",
           "mlp_train", "mlp_predict", "mlp_train_batched", "mlp_eval_batched", "mlp_cv_select",
           "mlp_shared_workspace_size",
           "mlp_train_shared", "mlp_train_shared_static", "mlp_barrier_probe", "mlp_set_momentum", "mlp_dense_forward", "mlp_dense_backward",
           "mlp_update", "mlp_mse_grad", "mlp_deep_train", "mlp_query_status", "mlp_workspace_status",
           "mlp_set_wait_limit", "mlp_mfma_probe", "mlp_set_launch_hint", "mlp_large_plan", "mlp_status_string",
           "mlp_last_error"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1908_07847_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    P = Params
    lib.mlp_workspace_size.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]
    lib.mlp_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Config), P, vp, vp, ctypes.c_size_t]
    lib.mlp_destroy.argtypes = [vp]
    lib.mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.mlp_backward.argtypes = [vp, vp, vp, vp, vp, vp, i64, P, vp, vp, vp]
    lib.mlp_step.argtypes = [vp, P, f32, vp]
    lib.mlp_train.argtypes = [vp, vp, vp, i32, vp, vp]
    lib.mlp_predict.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    lib.mlp_train_batched.argtypes = [ctypes.POINTER(BatchItem), vp, i32, i32, i32, vp, vp, i64, vp, vp,
                                      i64, i32, vp, vp]
    lib.mlp_eval_batched.argtypes = [ctypes.POINTER(BatchItem), vp, i32, i32, i32, vp, vp, i64, vp, i64, vp, vp,
                                     vp]
    lib.mlp_cv_select.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    lib.mlp_shared_workspace_size.argtypes = [ctypes.POINTER(Config), i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.mlp_train_shared.argtypes = [ctypes.POINTER(Config), i32, ctypes.POINTER(f32), vp, vp, vp, vp, i32, vp,
                                     vp, ctypes.c_size_t, vp]
    lib.mlp_train_shared_static.argtypes = [ctypes.POINTER(Config), i32, ctypes.POINTER(f32), vp, vp, vp, vp, i32,
                                            vp, vp]
    lib.mlp_set_launch_hint.argtypes = [ctypes.POINTER(LaunchHint)]
    lib.mlp_large_plan.argtypes = [ctypes.POINTER(Config), i32, i32, ctypes.POINTER(i32)]
    lib.mlp_barrier_probe.argtypes = [i32, i32, vp, ctypes.c_size_t, vp]
    lib.mlp_set_momentum.argtypes = [vp, f32, vp]
    lib.mlp_dense_forward.argtypes = [vp, i64, i32, i32, vp, vp, i32, vp, vp]
    lib.mlp_dense_backward.argtypes = [vp, vp, vp, i64, i32, i32, vp, i32, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.mlp_update.argtypes = [vp, vp, vp, i64, f32, vp]
    lib.mlp_mse_grad.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    lib.mlp_deep_train.argtypes = [vp, vp, i64, i32, ctypes.POINTER(i32), i32, vp, vp, f32, i32, vp, vp]
    lib.mlp_query_status.argtypes = [vp, vp]
    lib.mlp_workspace_status.argtypes = [vp, ctypes.c_size_t, vp]
    lib.mlp_set_wait_limit.argtypes = [i64]
    lib.mlp_mfma_probe.argtypes = [i32, vp, vp, vp, i32, i32, i32, vp]
    for name in SYMBOLS:
        if name not in ("mlp_status_string", "mlp_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    lib.mlp_status_string.argtypes = [ctypes.c_int]
    lib.mlp_status_string.restype = ctypes.c_char_p
    lib.mlp_last_error.argtypes = []
    lib.mlp_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def check(status: int) -> None:
    if status != MLP_OK:
        raise MLPError(status, lib.mlp_last_error().decode())
