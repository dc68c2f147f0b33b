"""Python binding of libniorca (the MI355X non-induced orbit counter).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libniorca.so`` behind the C ABI of ``include/niorca.h``.  Tensors
are torch CUDA (HIP) tensors; the library is called on torch's current stream.
There is no CPU path: if the library or a GPU is missing, calls raise.

    count(row_ptr, col)          -> int64[n, 15]   psi_k(x), k = 0..14
    count(..., flags=INDUCED)    -> int64[n, 15]   induced counts psi'_k(x)
    edge_triangles(row_ptr, col) -> int32[nnz]     Stage I, per input CSR slot
    edge_k4(row_ptr, col)        -> int64[nnz]     4-cliques through each edge
    k4(row_ptr, col)             -> int64[n]       Stage II
    fvars(row_ptr, col)          -> int64[n, 9]    Stage III-a (Table 1 order)
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libniorca.so")

OK, EINVAL, ENOTSIMPLE, EOVERFLOW, ENOMEM, EDEVICE, ENOTIMPL, EINTERNAL = range(8)
STATUS_NAMES = ["OK", "EINVAL", "ENOTSIMPLE", "EOVERFLOW", "ENOMEM", "EDEVICE", "ENOTIMPL", "EINTERNAL"]
VALIDATE, BIN_DEGREE, BIN_MLP, COUNTERS, TIMING, INDUCED = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
GRAPH_CAPTURE = 0x100
F_NAMES = ["f12_14", "f10_13", "f13_14", "f11_13", "f5_8", "f6_9", "f9_12", "f4_8", "f8_12"]

# Every symbol include/niorca.h declares (checked by the CPU tests).
EXPORTS = ["niorca_create", "niorca_destroy", "niorca_last_error", "niorca_set_workspace_limit",
           "niorca_workspace_bytes", "niorca_set_param", "niorca_count", "niorca_count_batched",
           "niorca_edge_triangles", "niorca_k4", "niorca_fvars", "niorca_work_counters",
           "niorca_set_cost_model", "niorca_stage_times", "niorca_last_features", "niorca_mlp_train",
           "niorca_mlp_predict", "niorca_kernel_times", "niorca_class_stats", "niorca_edge_k4",
           "niorca_device_status", "niorca_load_tuning", "niorca_count_noalloc"]
KERNEL_NAMES = ["probe_thread", "probe_wave", "probe_block", "probe_large", "ql_wave", "ql_block", "ql_global",
                "qh_wave", "qh_block", "qh_dense", "qh_global", "probe_group"]
CLASS_NAMES = ["tri_wave", "tri_thread", "tri_block", "tri_large", "ql_wave", "ql_block", "ql_global",
               "qh_wave", "qh_block", "qh_dense", "qh_global", "tri_group"]
NUM_COUNTERS = 7
MLP_PARAMS = 1325
COUNTER_NAMES = ["probes", "triangles", "k4_words", "wedges_light", "wedges_heavy", "sum_slots", "stage1_cycles"]
STAGE_NAMES = ["relabel", "setup", "orient", "zero", "stage1_k4", "sums", "tau", "cycles4", "solve"]


class NiorcaError(RuntimeError):
    def __init__(self, status: int, message: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")
        self.status = status


_lib = None
_lock = threading.Lock()
_ctx = {}


def load_library():
    """Load libniorca.so (never builds it; run build.build() or __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2606_29651_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        lib.niorca_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        lib.niorca_destroy.argtypes = [P]
        lib.niorca_destroy.restype = None
        lib.niorca_last_error.argtypes = [P]
        lib.niorca_last_error.restype = ctypes.c_char_p
        lib.niorca_set_workspace_limit.argtypes = [P, u64]
        lib.niorca_workspace_bytes.argtypes = [P]
        lib.niorca_workspace_bytes.restype = u64
        lib.niorca_set_param.argtypes = [P, ctypes.c_char_p, i64]
        lib.niorca_count.argtypes = [P, i32, i64, P, P, P, P, u32]
        lib.niorca_count_batched.argtypes = [P, i32, P, i64, P, P, P, P, u32]
        lib.niorca_count_noalloc.argtypes = [P, i32, i64, P, P, P, P, u32]
        lib.niorca_edge_triangles.argtypes = [P, i32, i64, P, P, P, P]
        lib.niorca_k4.argtypes = [P, i32, i64, P, P, P, P]
        lib.niorca_edge_k4.argtypes = [P, i32, i64, P, P, P, P]
        lib.niorca_device_status.argtypes = [P, P]
        lib.niorca_load_tuning.argtypes = [P, ctypes.c_char_p, ctypes.c_char_p]
        lib.niorca_fvars.argtypes = [P, i32, i64, P, P, P, P]
        lib.niorca_work_counters.argtypes = [P, i32, P, P]
        lib.niorca_set_cost_model.argtypes = [P, P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float]
        lib.niorca_stage_times.argtypes = [P, P, i32]
        lib.niorca_kernel_times.argtypes = [P, P, i32]
        lib.niorca_class_stats.argtypes = [P, P, i32]
        lib.niorca_last_features.argtypes = [P, i32, P, P]
        lib.niorca_mlp_train.argtypes = [P, P, P, i64, i32, i32, ctypes.c_float, u64, P, P, P]
        lib.niorca_mlp_predict.argtypes = [P, P, P, i64, P, P]
        for name in EXPORTS:
            if name not in ("niorca_destroy", "niorca_last_error", "niorca_workspace_bytes"):
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


class Context:
    """One library context (device workspace) on one device."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        rc = lib.niorca_create(ctypes.byref(h), int(device))
        if rc != OK:
            raise NiorcaError(rc, f"niorca_create(device={device})")
        self.h = h
        self.device = device
        self.lib = lib

    def close(self):
        if self.h:
            self.lib.niorca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, what: str):
        if rc != OK:
            msg = self.lib.niorca_last_error(self.h).decode()
            raise NiorcaError(rc, f"{what}: {msg}")

    def set_param(self, name: str, value: int):
        self.check(self.lib.niorca_set_param(self.h, name.encode(), int(value)), f"set_param({name})")

    def load_tuning(self, path: str, key: str):
        """Apply the knobs stored under key in a tuning file (niorca_load_tuning)."""
        self.check(self.lib.niorca_load_tuning(self.h, path.encode(), key.encode()), f"load_tuning({key})")

    def device_status(self, stream=None):
        """Wait for the last call on this context and raise if its kernels flagged bad
        input rows or an odd halved numerator (niorca_device_status)."""
        self.check(self.lib.niorca_device_status(self.h, _stream_ptr(stream)), "niorca_device_status")

    def set_workspace_limit(self, nbytes: int):
        self.check(self.lib.niorca_set_workspace_limit(self.h, int(nbytes)), "set_workspace_limit")

    def workspace_bytes(self) -> int:
        return int(self.lib.niorca_workspace_bytes(self.h))

    def kernel_times(self) -> dict:
        """Per-kernel ms of the last call made with TIMING (waits for it)."""
        buf = (ctypes.c_float * len(KERNEL_NAMES))()
        self.check(self.lib.niorca_kernel_times(self.h, ctypes.cast(buf, ctypes.c_void_p), len(KERNEL_NAMES)),
                   "kernel_times")
        return dict(zip(KERNEL_NAMES, [float(x) for x in buf]))

    def class_stats(self) -> dict:
        """{class: (vertices, work units, row slots)} of the last count."""
        import numpy as np
        k = len(CLASS_NAMES)
        buf = np.zeros(3 * k, dtype=np.int64)
        self.check(self.lib.niorca_class_stats(self.h, buf.ctypes.data_as(ctypes.c_void_p), 3 * k), "class_stats")
        return {name: (int(buf[i]), int(buf[k + i]), int(buf[2 * k + i])) for i, name in enumerate(CLASS_NAMES)}

    def stage_times(self) -> dict:
        """Per-stage ms of the last call made with TIMING (waits for it)."""
        buf = (ctypes.c_float * len(STAGE_NAMES))()
        self.check(self.lib.niorca_stage_times(self.h, ctypes.cast(buf, ctypes.c_void_p), len(STAGE_NAMES)),
                   "stage_times")
        return dict(zip(STAGE_NAMES, [float(x) for x in buf]))


def context(device=None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    with _lock:
        c = _ctx.get(device)
        if c is None:
            c = Context(device)
            _ctx[device] = c
        return c


def _graph(row_ptr: torch.Tensor, col: torch.Tensor):
    if not (row_ptr.is_cuda and col.is_cuda):
        raise ValueError("row_ptr and col must be device tensors")
    if row_ptr.dtype != torch.int64 or col.dtype != torch.int32:
        raise TypeError("row_ptr must be int64 and col int32")
    row_ptr = row_ptr.contiguous()
    col = col.contiguous()
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr needs n+1 entries")
    return row_ptr, col, n, col.numel()


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _p(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def count(row_ptr: torch.Tensor, col: torch.Tensor, flags: int = 0, out: torch.Tensor = None,
          ctx: Context = None, stream=None) -> torch.Tensor:
    """psi[x, k] (int64[n, 15]) for the graph in device CSR (row_ptr int64, col int32)."""
    row_ptr, col, n, nnz = _graph(row_ptr, col)
    ctx = ctx or context(row_ptr.device.index)
    if out is None:
        out = torch.empty((n, 15), dtype=torch.int64, device=row_ptr.device)
    ctx.check(ctx.lib.niorca_count(ctx.h, n, nnz, _p(row_ptr), _p(col), _p(out), _stream_ptr(stream), flags),
              "niorca_count")
    return out


def count_noalloc(row_ptr: torch.Tensor, col: torch.Tensor, out: torch.Tensor, flags: int = 0,
                  ctx: Context = None, stream=None) -> torch.Tensor:
    """count() into a caller-provided out (int64[n, 15]) with the library's fixed
    device scratch as workspace: no device allocation in the call."""
    row_ptr, col, n, nnz = _graph(row_ptr, col)
    ctx = ctx or context(row_ptr.device.index)
    if out.dtype != torch.int64 or out.shape != (n, 15) or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 tensor of shape (n, 15)")
    ctx.check(ctx.lib.niorca_count_noalloc(ctx.h, n, nnz, _p(row_ptr), _p(col), _p(out), _stream_ptr(stream),
                                           flags), "niorca_count_noalloc")
    return out


def edge_triangles(row_ptr, col, ctx: Context = None, stream=None) -> torch.Tensor:
    row_ptr, col, n, nnz = _graph(row_ptr, col)
    ctx = ctx or context(row_ptr.device.index)
    tri = torch.empty(nnz, dtype=torch.int32, device=row_ptr.device)
    ctx.check(ctx.lib.niorca_edge_triangles(ctx.h, n, nnz, _p(row_ptr), _p(col), _p(tri), _stream_ptr(stream)),
              "niorca_edge_triangles")
    return tri


def k4(row_ptr, col, ctx: Context = None, stream=None) -> torch.Tensor:
    row_ptr, col, n, nnz = _graph(row_ptr, col)
    ctx = ctx or context(row_ptr.device.index)
    out = torch.empty(n, dtype=torch.int64, device=row_ptr.device)
    ctx.check(ctx.lib.niorca_k4(ctx.h, n, nnz, _p(row_ptr), _p(col), _p(out), _stream_ptr(stream)), "niorca_k4")
    return out


def edge_k4(row_ptr, col, ctx: Context = None, stream=None) -> torch.Tensor:
    """int64[nnz]: the number of 4-cliques through the edge of each input CSR slot."""
    row_ptr, col, n, nnz = _graph(row_ptr, col)
    ctx = ctx or context(row_ptr.device.index)
    out = torch.empty(nnz, dtype=torch.int64, device=row_ptr.device)
    ctx.check(ctx.lib.niorca_edge_k4(ctx.h, n, nnz, _p(row_ptr), _p(col), _p(out), _stream_ptr(stream)),
              "niorca_edge_k4")
    return out


def fvars(row_ptr, col, ctx: Context = None, stream=None) -> torch.Tensor:
    row_ptr, col, n, nnz = _graph(row_ptr, col)
    ctx = ctx or context(row_ptr.device.index)
    out = torch.empty((n, 9), dtype=torch.int64, device=row_ptr.device)
    ctx.check(ctx.lib.niorca_fvars(ctx.h, n, nnz, _p(row_ptr), _p(col), _p(out), _stream_ptr(stream)),
              "niorca_fvars")
    return out


def count_batched(vtx_off, row_ptr: torch.Tensor, col: torch.Tensor, flags: int = 0, out: torch.Tensor = None,
                  ctx: Context = None, stream=None) -> torch.Tensor:
    """psi (int64[total_n, 15]) of many packed graphs: vtx_off is a host int64 array
    (numpy or list), row_ptr global, col ids local to each graph."""
    import numpy as np
    voff = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    row_ptr, col, n, nnz = _graph(row_ptr, col)
    if voff.ndim != 1 or voff.shape[0] < 1 or int(voff[-1]) != n:
        raise ValueError("vtx_off must end at the number of rows")
    ctx = ctx or context(row_ptr.device.index)
    if out is None:
        out = torch.empty((n, 15), dtype=torch.int64, device=row_ptr.device)
    rc = ctx.lib.niorca_count_batched(ctx.h, voff.shape[0] - 1, voff.ctypes.data_as(ctypes.c_void_p), nnz,
                                      _p(row_ptr), _p(col), _p(out), _stream_ptr(stream), flags)
    ctx.check(rc, "niorca_count_batched")
    return out


def work_counters(n: int, ctx: Context = None, device=None, stream=None) -> torch.Tensor:
    """int64[n, 7] work counters of the last count made with COUNTERS on ctx."""
    ctx = ctx or context(device)
    out = torch.empty((n, NUM_COUNTERS), dtype=torch.int64, device=f"cuda:{ctx.device}")
    ctx.check(ctx.lib.niorca_work_counters(ctx.h, n, _p(out), _stream_ptr(stream)), "niorca_work_counters")
    return out


def last_features(n: int, ctx: Context = None, device=None, stream=None) -> torch.Tensor:
    """float32[n, 6] features of the last count made with COUNTERS or BIN_MLP on ctx."""
    ctx = ctx or context(device)
    out = torch.empty((n, 6), dtype=torch.float32, device=f"cuda:{ctx.device}")
    ctx.check(ctx.lib.niorca_last_features(ctx.h, n, _p(out), _stream_ptr(stream)), "niorca_last_features")
    return out


def mlp_train(X: torch.Tensor, y: torch.Tensor, epochs: int = 8, batch: int = 4096, lr: float = 3e-3,
              seed: int = 1, ctx: Context = None, stream=None):
    """Train the work model on device features X[N, 6] and targets y[N]; returns
    (model as a numpy float32[1325], final mean squared error)."""
    import numpy as np
    X = X.contiguous().float()
    y = y.contiguous().float()
    ctx = ctx or context(X.device.index)
    model = np.zeros(MLP_PARAMS, dtype=np.float32)
    mse = ctypes.c_double()
    rc = ctx.lib.niorca_mlp_train(ctx.h, _p(X), _p(y), X.shape[0], epochs, batch, lr, seed,
                                  model.ctypes.data_as(ctypes.c_void_p), ctypes.byref(mse), _stream_ptr(stream))
    ctx.check(rc, "niorca_mlp_train")
    return model, mse.value


def mlp_predict(model, X: torch.Tensor, ctx: Context = None, stream=None) -> torch.Tensor:
    import numpy as np
    model = np.ascontiguousarray(model, dtype=np.float32)
    X = X.contiguous().float()
    ctx = ctx or context(X.device.index)
    out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    ctx.check(ctx.lib.niorca_mlp_predict(ctx.h, model.ctypes.data_as(ctypes.c_void_p), _p(X), X.shape[0], _p(out),
                                         _stream_ptr(stream)), "niorca_mlp_predict")
    return out


def set_cost_model(model, thr_thread: float, thr_block: float, thr_group: float = None, ctx: Context = None,
                   device=None):
    """Load the work model for BIN_MLP with its thresholds on predicted log2 work:
    one lane up to thr_thread, sixteen lanes up to thr_group (None: no such class),
    a workgroup from thr_block."""
    import numpy as np
    model = np.ascontiguousarray(model, dtype=np.float32)
    if model.shape != (MLP_PARAMS,):
        raise ValueError(f"model must hold {MLP_PARAMS} floats")
    ctx = ctx or context(device)
    ctx.check(ctx.lib.niorca_set_cost_model(ctx.h, model.ctypes.data_as(ctypes.c_void_p), MLP_PARAMS,
                                            float(thr_thread), float(-1e30 if thr_group is None else thr_group),
                                            float(thr_block)), "niorca_set_cost_model")
