"""ctypes binding of libf2v.so (include/f2v.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  Device buffers are torch CUDA (HIP) tensors; the library works on
the tensors' memory and on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libf2v.so")

# Names declared in include/f2v.h (the CPU tests check they are all exported).
EXPORTS = (
    "f2v_default_params", "f2v_workspace_size", "f2v_init", "f2v_epoch", "f2v_loss",
    "f2v_sync_embedding", "f2v_check", "f2v_destroy", "f2v_status_string", "f2v_last_error",
    "f2v_partition", "f2v_negatives", "f2v_last_epoch_ms", "f2v_set_diagnostics", "f2v_wave_stats",
    "f2v_vertex_trace", "f2v_footprint", "f2v_server_create", "f2v_server_submit",
    "f2v_server_flush", "f2v_server_poll", "f2v_server_query", "f2v_server_drain",
    "f2v_server_destroy", "f2v_server_last_error", "f2v_random_embedding", "f2v_health",
    "f2v_walks", "f2v_step_size", "f2v_train_static", "f2v_selftest_publish", "f2v_server_health",
)

STATUS = {0: "F2V_OK", 1: "F2V_E_INVALID_ARG", 2: "F2V_E_BAD_GRAPH", 3: "F2V_E_OOM", 4: "F2V_E_HIP",
          5: "F2V_E_STATE", 6: "F2V_E_TIMEOUT", 7: "F2V_E_BUSY", 8: "F2V_E_UNSUPPORTED"}
FORCE = {"sigmoid": 0, "student_t": 1, "fr": 2, "linlog": 3, "forceatlas": 4}
PRECISION = {"fp32": 0, "bf16": 1}
LR_SCHEDULE = {"const": 0, "linear": 1}
PERM = {"random": 0, "identity": 1}
SCHEDULE = {"dataflow": 0, "strict": 1, "dynamic": 2, "hogwild": 3}


class F2VError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Params(ctypes.Structure):
    """Mirror of f2v_params."""
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("d", ctypes.c_int32),
        ("batch", ctypes.c_int32), ("s", ctypes.c_int32), ("force", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("lr_schedule", ctypes.c_int32), ("lr0", ctypes.c_float),
        ("eps", ctypes.c_float), ("total_epochs", ctypes.c_int32), ("perm_mode", ctypes.c_int32),
        ("schedule", ctypes.c_int32), ("chunk", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("late_window", ctypes.c_int32), ("fan_in", ctypes.c_int32), ("walk_length", ctypes.c_int32),
        ("stage_negatives", ctypes.c_int32),
    ]


_lib = None


def load(build_if_missing: bool = True):
    """Load libf2v.so (building it first if it is not there)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise ImportError(f"{LIB_PATH} is not built")
        from . import build as _build
        _build.build()
    L = ctypes.CDLL(LIB_PATH)
    P, st = ctypes.c_void_p, ctypes.c_int
    PP = ctypes.POINTER(Params)
    L.f2v_default_params.argtypes = [PP]
    L.f2v_default_params.restype = None
    L.f2v_workspace_size.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
    L.f2v_workspace_size.restype = st
    L.f2v_init.argtypes = [PP, P, P, P, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.f2v_init.restype = st
    L.f2v_epoch.argtypes = [P, ctypes.c_int32]
    L.f2v_epoch.restype = st
    L.f2v_loss.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    L.f2v_loss.restype = st
    for name in ("f2v_sync_embedding", "f2v_check", "f2v_destroy"):
        getattr(L, name).argtypes = [P]
        getattr(L, name).restype = st
    L.f2v_status_string.argtypes = [st]
    L.f2v_status_string.restype = ctypes.c_char_p
    L.f2v_last_error.argtypes = [P]
    L.f2v_last_error.restype = ctypes.c_char_p
    L.f2v_partition.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, P, P]
    L.f2v_partition.restype = st
    L.f2v_negatives.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                ctypes.c_int32, P, P]
    L.f2v_negatives.restype = st
    L.f2v_last_epoch_ms.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    L.f2v_last_epoch_ms.restype = st
    L.f2v_set_diagnostics.argtypes = [P, ctypes.c_int32]
    L.f2v_set_diagnostics.restype = st
    L.f2v_wave_stats.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.f2v_wave_stats.restype = st
    L.f2v_vertex_trace.argtypes = [P, P]
    L.f2v_vertex_trace.restype = st
    L.f2v_footprint.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
    L.f2v_footprint.restype = st
    L.f2v_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(P)]
    L.f2v_server_create.restype = st
    L.f2v_server_submit.argtypes = [P, PP, P, P, P, P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_uint64)]
    L.f2v_server_submit.restype = st
    for name in ("f2v_server_flush", "f2v_server_drain", "f2v_server_destroy"):
        getattr(L, name).argtypes = [P]
        getattr(L, name).restype = st
    L.f2v_server_poll.argtypes = [P, P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.f2v_server_poll.restype = st
    L.f2v_server_query.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    L.f2v_server_query.restype = st
    L.f2v_server_health.argtypes = [P, ctypes.POINTER(ctypes.c_uint64)]
    L.f2v_server_health.restype = st
    L.f2v_random_embedding.argtypes = [P, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float, P]
    L.f2v_random_embedding.restype = st
    L.f2v_walks.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, P, P, P]
    L.f2v_walks.restype = st
    L.f2v_selftest_publish.argtypes = [ctypes.c_int32, ctypes.c_int32, P, ctypes.c_size_t,
                                       ctypes.POINTER(ctypes.c_uint32), P]
    L.f2v_selftest_publish.restype = st
    L.f2v_train_static.argtypes = [PP, P, P, P, ctypes.c_int32, ctypes.c_int32, P]
    L.f2v_train_static.restype = st
    L.f2v_step_size.argtypes = [PP, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]
    L.f2v_step_size.restype = st
    L.f2v_health.argtypes = [P, P, ctypes.POINTER(ctypes.c_int32)]
    L.f2v_health.restype = st
    L.f2v_server_last_error.argtypes = [P]
    L.f2v_server_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int, ctx=None) -> None:
    if status != 0:
        msg = load().f2v_last_error(ctx).decode(errors="replace")
        raise F2VError(status, msg)


def make_params(n: int, nnz: int, d: int, *, batch: int = 384, s: int = 5, force: str = "sigmoid",
                precision: str = "fp32", lr0: float = 0.02, lr_schedule: str = "const",
                eps: float = 1e-3, total_epochs: int = 1, perm_mode: str = "random",
                schedule: str = "dataflow", chunk: int | None = None, seed: int = 0,
                late_window: int | None = None, fan_in: int | None = None, walk_length: int = 0,
                stage_negatives: int = 0) -> Params:
    p = Params()
    load().f2v_default_params(ctypes.byref(p))
    p.n, p.nnz, p.d, p.batch, p.s = n, nnz, d, batch, s
    p.force = FORCE[force]
    p.precision = PRECISION[precision]
    p.lr0, p.lr_schedule, p.eps = lr0, LR_SCHEDULE[lr_schedule], eps
    p.total_epochs, p.perm_mode, p.schedule = total_epochs, PERM[perm_mode], SCHEDULE[schedule]
    if chunk:
        p.chunk = chunk
    p.seed = seed
    if late_window is not None:
        p.late_window = late_window
    if fan_in is not None:
        p.fan_in = fan_in
    p.walk_length = walk_length
    p.stage_negatives = stage_negatives
    return p


def footprint(p: Params) -> int:
    """Device bytes of one job: CSR, embedding and workspace."""
    out = ctypes.c_size_t(0)
    check(load().f2v_footprint(ctypes.byref(p), ctypes.byref(out)))
    return int(out.value)


def workspace_size(p: Params) -> int:
    out = ctypes.c_size_t(0)
    check(load().f2v_workspace_size(ctypes.byref(p), ctypes.byref(out)))
    return int(out.value)
