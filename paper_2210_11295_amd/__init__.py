"""Python binding of the gfx950 block SRHT library (libbsrht.so).

Thin ctypes marshalling over the C ABI of include/bsrht.h: the same names,
torch tensors for device memory and torch's current HIP stream by default.
Every step of the sketch, the randomized SVD and the Nystrom method runs in
the library's HIP kernels; this module only allocates buffers and passes
pointers.  It raises if the library has not been built; there is no other
execution path.
"""

import atexit
import ctypes
import os

import numpy as np
import torch

__all__ = [
    "BsrhtError", "lib", "library_path", "Plan", "bsrht_plan_bytes", "bsrht_plan",
    "bsrht_apply", "bsrht_apply_workspace", "rsvd", "rsvd_workspace", "nystrom",
    "nystrom_workspace", "WITH_REPLACEMENT", "WITHOUT_REPLACEMENT", "FP32",
    "SPLIT_BF16", "INFO_CHOL_FALLBACK", "INFO_RANK_CLAMPED", "INFO_QB_FALLBACK",
    "INFO_JACOBI_NOCONV", "EXPORTED_SYMBOLS", "JOB_SKETCH", "JOB_RSVD", "JOB_NYSTROM", "JobDesc",
    "JobResult", "ServerStats", "Server", "bsrht_job_bytes", "apply_batch",
    "batch_table_bytes", "ApplyItem", "BATCH_MAX", "bsrht_apply_right",
    "bsrht_apply_right_workspace", "rsvd_single_view", "rsvd_single_view_workspace",
    "bsrht_dense_sketch", "bsrht_dense_workspace", "DENSE_GAUSSIAN", "DENSE_RADEMACHER",
    "nystrom_shifted", "nystrom_job", "finalize", "Task", "rsvd_start", "nystrom_start",
    "rsvd_single_view_start",
]

WITH_REPLACEMENT = 0
WITHOUT_REPLACEMENT = 1
FP32 = 0
SPLIT_BF16 = 1
INFO_CHOL_FALLBACK = 1
INFO_RANK_CLAMPED = 2
INFO_QB_FALLBACK = 4
INFO_JACOBI_NOCONV = 8
TIMING_OFF = 0
TIMING_APPLY_FP32 = 1
TIMING_APPLY_BF16 = 2
TIMING_GEMM_AQ = 3
TIMING_STREAM = 4
TIMING_APPLY_RIGHT = 5
TIMING_DENSE_GEMM = 6
DENSE_GAUSSIAN = 0
DENSE_RADEMACHER = 1
STREAM_BLOCKS = 4096
JOB_SKETCH = 0
JOB_RSVD = 1
JOB_NYSTROM = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "_lib", "libbsrht.so")

_c_i64 = ctypes.c_int64
_c_vp = ctypes.c_void_p
_c_sz = ctypes.c_size_t

# name -> (restype, argtypes); the declarations of include/bsrht.h
_SIGS = {
    "bsrht_version": (ctypes.c_char_p, []),
    "bsrht_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "bsrht_plan_bytes": (_c_sz, [_c_i64, _c_i64, _c_i64]),
    "bsrht_plan": (ctypes.c_int, [_c_i64, _c_i64, _c_i64, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_int, _c_vp, _c_sz, _c_vp, ctypes.POINTER(_c_vp)]),
    "bsrht_plan_destroy": (ctypes.c_int, [_c_vp]),
    "bsrht_plan_info": (ctypes.c_int, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp]),
    "bsrht_plan_export": (ctypes.c_int, [_c_vp, _c_vp, _c_vp, _c_vp]),
    "bsrht_apply_workspace": (_c_sz, [_c_vp, _c_i64]),
    "bsrht_apply": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_vp, _c_i64, _c_vp,
                                   _c_sz, _c_vp]),
    "bsrht_apply_noalloc": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_vp, _c_i64,
                                           _c_vp]),
    "bsrht_apply_right_workspace": (_c_sz, [_c_vp, _c_i64]),
    "bsrht_apply_right": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_vp, _c_i64, _c_vp,
                                         _c_sz, _c_vp]),
    "rsvd_workspace": (_c_sz, [_c_vp, _c_i64, _c_i64]),
    "rsvd": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_i64, _c_vp, _c_vp, _c_vp,
                            _c_vp, _c_vp, _c_sz, _c_vp]),
    "nystrom_workspace": (_c_sz, [_c_vp, _c_i64]),
    "rsvd_single_view_workspace": (_c_sz, [_c_vp, _c_vp, _c_vp, _c_vp, _c_i64]),
    "bsrht_dense_workspace": (_c_sz, [_c_i64, _c_i64, _c_i64]),
    "bsrht_dense_sketch": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, _c_i64, _c_i64, _c_vp,
                                          _c_i64, _c_i64, _c_vp, _c_i64, _c_vp, _c_sz, _c_vp]),
    "rsvd_single_view": (ctypes.c_int, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_i64, _c_i64,
                                        _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_sz, _c_vp]),
    "bsrht_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "bsrht_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(_c_i64)]),
    "bsrht_timing_samples": (ctypes.c_int, [_c_vp, _c_i64, ctypes.POINTER(_c_i64)]),
    "bsrht_batch_table_bytes": (_c_sz, []),
    "bsrht_apply_batch": (ctypes.c_int, [_c_vp, ctypes.c_int, _c_vp, _c_sz, _c_vp]),
    "bsrht_stream_read": (ctypes.c_int, [_c_vp, _c_i64, _c_vp, _c_vp]),
    "bsrht_batch_table_release": (ctypes.c_int, [_c_vp]),
    "bsrht_finalize": (ctypes.c_int, []),
    "nystrom": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp,
                               _c_sz, _c_vp]),
    "nystrom_shifted": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_vp, _c_vp, _c_vp,
                                       _c_vp, _c_sz, _c_vp]),
    "rsvd_start": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_i64, _c_vp, _c_vp, _c_vp,
                                  _c_vp, _c_vp, _c_sz, _c_vp, ctypes.POINTER(_c_vp)]),
    "nystrom_start": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp,
                                     _c_sz, _c_vp, ctypes.POINTER(_c_vp)]),
    "nystrom_shifted_start": (ctypes.c_int, [_c_vp, _c_vp, _c_i64, _c_i64, _c_vp, _c_vp, _c_vp,
                                             _c_vp, _c_sz, _c_vp, ctypes.POINTER(_c_vp)]),
    "rsvd_single_view_start": (ctypes.c_int, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_i64, _c_i64,
                                              _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_sz, _c_vp,
                                              ctypes.POINTER(_c_vp)]),
    "bsrht_task_poll": (ctypes.c_int, [_c_vp, ctypes.POINTER(ctypes.c_int)]),
    "bsrht_task_wait": (ctypes.c_int, [_c_vp]),
    "bsrht_task_destroy": (ctypes.c_int, [_c_vp]),
}


class JobDesc(ctypes.Structure):
    """bsrht_job_t of include/bsrht_serve.h."""
    _fields_ = [("id", _c_i64), ("kind", ctypes.c_int), ("n", _c_i64), ("m", _c_i64),
                ("p", _c_i64), ("l", _c_i64), ("k", _c_i64), ("seed", ctypes.c_uint64),
                ("sampling", ctypes.c_int), ("precision", ctypes.c_int), ("A", _c_vp),
                ("lda", _c_i64), ("Y", _c_vp), ("ldy", _c_i64), ("U", _c_vp), ("S", _c_vp),
                ("V", _c_vp), ("info", _c_vp)]


class JobResult(ctypes.Structure):
    """bsrht_job_result_t of include/bsrht_serve.h."""
    _fields_ = [("id", _c_i64), ("status", ctypes.c_int), ("arena_bytes", _c_i64),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    """bsrht_server_stats_t of include/bsrht_serve.h."""
    _fields_ = [("submitted", _c_i64), ("completed", _c_i64), ("rejected", _c_i64),
                ("plan_hits", _c_i64), ("plan_misses", _c_i64), ("plan_evictions", _c_i64),
                ("backfilled", _c_i64), ("peak_arena_bytes", _c_i64),
                ("peak_running", ctypes.c_int), ("queued", _c_i64),
                ("batches", _c_i64), ("batched_jobs", _c_i64)]


# the declarations of include/bsrht_serve.h
_SIGS.update({
    "bsrht_job_bytes": (_c_sz, [ctypes.POINTER(JobDesc)]),
    "bsrht_server_create": (ctypes.c_int, [_c_vp, _c_sz, ctypes.c_int, ctypes.POINTER(_c_vp)]),
    "bsrht_server_create_fake": (ctypes.c_int, [_c_sz, ctypes.c_int, ctypes.c_double,
                                                ctypes.POINTER(_c_vp)]),
    "bsrht_server_submit": (ctypes.c_int, [_c_vp, ctypes.POINTER(JobDesc)]),
    "bsrht_server_set_batching": (ctypes.c_int, [_c_vp, ctypes.c_int]),
    "bsrht_server_submit_many": (ctypes.c_int, [_c_vp, ctypes.POINTER(JobDesc), ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int)]),
    "bsrht_server_poll": (ctypes.c_int, [_c_vp, ctypes.POINTER(JobResult), ctypes.c_int,
                                         ctypes.c_double, ctypes.POINTER(ctypes.c_int)]),
    "bsrht_server_drain": (ctypes.c_int, [_c_vp]),
    "bsrht_server_stats": (ctypes.c_int, [_c_vp, ctypes.POINTER(ServerStats)]),
    "bsrht_server_clock": (ctypes.c_double, [_c_vp]),
    "bsrht_server_destroy": (ctypes.c_int, [_c_vp]),
})
EXPORTED_SYMBOLS = tuple(_SIGS)

_lib = None


class BsrhtError(RuntimeError):
    def __init__(self, fn, status):
        msg = lib().bsrht_strerror(status).decode()
        super().__init__(f"{fn} failed: {msg} ({status})")
        self.status = status


def lib():
    """The loaded libbsrht.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError(
                f"{library_path} is missing: build it with __graft_entry__.build() "
                "(hipcc for gfx950); there is no fallback path")
        handle = ctypes.CDLL(library_path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
        # release the library's process-lifetime HIP objects (batch graphs,
        # pinned staging, events) while the HIP runtime is still up
        atexit.register(_finalize)
    return _lib


def _finalize():
    if _lib is not None:
        _lib.bsrht_finalize()


def _check(fn, status):
    if status != 0:
        raise BsrhtError(fn, status)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_matrix(name, t, dtype=torch.float32):
    if not isinstance(t, torch.Tensor) or t.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if not t.is_cuda or t.dtype != dtype:
        raise ValueError(f"{name} must be a {dtype} tensor on a GPU")
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError(f"{name} must be row-major (unit column stride)")


def timing_enable(which):
    """Record HIP events around every launch of one library kernel (0 = off)."""
    _check("bsrht_timing_enable", lib().bsrht_timing_enable(which))


def timing_read():
    """(summed kernel milliseconds, launches) since timing_enable."""
    ms = ctypes.c_double()
    n = _c_i64()
    _check("bsrht_timing_read", lib().bsrht_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def timing_samples(cap=100000):
    """Per-launch kernel milliseconds (launch order) since timing_enable."""
    buf = (ctypes.c_float * max(cap, 1))()
    n = _c_i64()
    _check("bsrht_timing_samples", lib().bsrht_timing_samples(buf, cap, ctypes.byref(n)))
    return [float(buf[i]) for i in range(min(n.value, cap))]


def stream_read(x, out=None, stream=None):
    """Read-bandwidth reference: one pass over the contiguous float32 device
    tensor x; returns the per-workgroup partial sums (STREAM_BLOCKS floats)."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32 \
            or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 tensor on a GPU")
    if out is None:
        out = torch.empty(STREAM_BLOCKS, dtype=torch.float32, device=x.device)
    _check("bsrht_stream_read", lib().bsrht_stream_read(_ptr(x), x.numel(), _ptr(out),
                                                        _stream_ptr(stream)))
    return out


def bsrht_plan_bytes(n, p, l):
    return int(lib().bsrht_plan_bytes(n, p, l))


class Plan:
    """A block SRHT Omega (l x n, p blocks): device tables + library handle."""

    def __init__(self, n, p, l, seed, sampling=WITH_REPLACEMENT, precision=FP32,
                 device=None, stream=None):
        L = lib()
        nbytes = L.bsrht_plan_bytes(n, p, l)
        if nbytes == 0:
            raise ValueError(f"invalid block SRHT sizes n={n} p={p} l={l}")
        dev = torch.device(device) if device is not None else torch.device("cuda")
        self.tables = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        self.n, self.p, self.l, self.r = int(n), int(p), int(l), int(n) // int(p)
        self.rp = 1 << (self.r - 1).bit_length()  # block size padded to a power of two
        self.seed, self.sampling, self.precision = int(seed), int(sampling), int(precision)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.tables.device):
            st = L.bsrht_plan(n, p, l, ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), sampling,
                              precision, _ptr(self.tables), nbytes, _stream_ptr(stream),
                              ctypes.byref(h))
        _check("bsrht_plan", st)
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.bsrht_plan_destroy(h)
            self.handle = None

    def export(self):
        """(R int32[l], Dbits uint32[ceil(p*rp/32)], Dtbits uint32[p*ceil(l/32)])."""
        R = np.zeros(self.l, dtype=np.int32)
        Db = np.zeros((self.p * self.rp + 31) // 32, dtype=np.uint32)
        Dtb = np.zeros(self.p * ((self.l + 31) // 32), dtype=np.uint32)
        _check("bsrht_plan_export", lib().bsrht_plan_export(
            self.handle, R.ctypes.data_as(_c_vp), Db.ctypes.data_as(_c_vp),
            Dtb.ctypes.data_as(_c_vp)))
        return R, Db, Dtb


def bsrht_plan(n, p, l, seed, sampling=WITH_REPLACEMENT, precision=FP32, device=None,
               stream=None):
    return Plan(n, p, l, seed, sampling, precision, device, stream)


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def bsrht_apply_workspace(plan, m):
    return int(lib().bsrht_apply_workspace(plan.handle, m))


def bsrht_apply(plan, A, Y=None, ws=None, stream=None):
    """Y = Omega A for a row-major float32 n x m device tensor A."""
    _check_matrix("A", A)
    n, m = A.shape
    if n != plan.n:
        raise ValueError(f"A has {n} rows, the plan expects {plan.n}")
    if Y is None:
        Y = torch.empty(plan.l, m, dtype=torch.float32, device=A.device)
    _check_matrix("Y", Y)
    need = bsrht_apply_workspace(plan, m)
    if ws is None:
        ws = _workspace(need, A.device)
    _check("bsrht_apply", lib().bsrht_apply(
        plan.handle, _ptr(A), m, max(A.stride(0), m), _ptr(Y), max(Y.stride(0), m),
        _ptr(ws), ws.numel(), _stream_ptr(stream)))
    return Y


NOALLOC_SCRATCH_BYTES = 32 << 20


def bsrht_apply_noalloc(plan, A, Y, stream=None):
    """Y = Omega A through the allocation-free entry point (the partials in
    the library's per-device scratch array; Y is the caller's)."""
    _check_matrix("A", A)
    n, m = A.shape
    if n != plan.n:
        raise ValueError(f"A has {n} rows, the plan expects {plan.n}")
    _check_matrix("Y", Y)
    _check("bsrht_apply_noalloc", lib().bsrht_apply_noalloc(
        plan.handle, _ptr(A), m, max(A.stride(0), m), _ptr(Y), max(Y.stride(0), m),
        _stream_ptr(stream)))
    return Y


def bsrht_apply_right_workspace(plan, m):
    return int(lib().bsrht_apply_right_workspace(plan.handle, m))


def bsrht_apply_right(plan, A, Y=None, ws=None, stream=None):
    """Y = A Omega^T for a row-major float32 m x n device tensor A (Y: m x l)."""
    _check_matrix("A", A)
    m, n = A.shape
    if n != plan.n:
        raise ValueError(f"A has {n} columns, the plan expects {plan.n}")
    if Y is None:
        Y = torch.empty(m, plan.l, dtype=torch.float32, device=A.device)
    _check_matrix("Y", Y)
    if tuple(Y.shape) != (m, plan.l):
        raise ValueError(f"Y must be {m} x {plan.l}")
    need = bsrht_apply_right_workspace(plan, m)
    if ws is None:
        ws = _workspace(need, A.device)
    _check("bsrht_apply_right", lib().bsrht_apply_right(
        plan.handle, _ptr(A), m, max(A.stride(0), n), _ptr(Y), max(Y.stride(0), plan.l),
        _ptr(ws), ws.numel(), _stream_ptr(stream)))
    return Y


BATCH_MAX = 64


class ApplyItem(ctypes.Structure):
    """bsrht_apply_item_t of include/bsrht.h: one bsrht_apply argument set."""
    _fields_ = [("plan", _c_vp), ("A", _c_vp), ("m", _c_i64), ("lda", _c_i64),
                ("Y", _c_vp), ("ldy", _c_i64), ("ws", _c_vp), ("ws_bytes", _c_sz)]


def batch_table_bytes():
    return int(lib().bsrht_batch_table_bytes())


def apply_batch(items, table, stream=None):
    """Several FP32 sketches in one persistent, graph-replayed launch.

    items: sequence of (plan, A, Y, ws) with bsrht_apply's meaning (ws of at
    least bsrht_apply_workspace(plan, m) bytes); table: a device uint8 tensor
    of batch_table_bytes() bytes.  Each Y is bitwise what bsrht_apply gives."""
    arr = (ApplyItem * max(len(items), 1))()
    for i, (plan, A, Y, ws) in enumerate(items):
        _check_matrix("A", A)
        _check_matrix("Y", Y)
        n, m = A.shape
        if n != plan.n or Y.shape[0] != plan.l or Y.shape[1] != m:
            raise ValueError("item shapes do not match its plan")
        arr[i] = ApplyItem(plan.handle.value if isinstance(plan.handle, ctypes.c_void_p)
                           else plan.handle, A.data_ptr(), m, max(A.stride(0), m),
                           Y.data_ptr(), max(Y.stride(0), m),
                           ws.data_ptr() if ws is not None and ws.numel() else None,
                           ws.numel() if ws is not None else 0)
    _check("bsrht_apply_batch", lib().bsrht_apply_batch(
        arr, len(items), _ptr(table), table.numel(), _stream_ptr(stream)))


def rsvd_workspace(plan, m, k):
    return int(lib().rsvd_workspace(plan.handle, m, k))


def rsvd(plan, A, k, ws=None, stream=None):
    """Randomized SVD (Algorithm 1 on A^T): returns (U n x k, S k float64, V m x k, info)."""
    _check_matrix("A", A)
    n, m = A.shape
    if n != plan.n:
        raise ValueError(f"A has {n} rows, the plan expects {plan.n}")
    dev = A.device
    U = torch.empty(n, k, dtype=torch.float32, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty(m, k, dtype=torch.float32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = _workspace(rsvd_workspace(plan, m, k), dev)
    _check("rsvd", lib().rsvd(plan.handle, _ptr(A), m, max(A.stride(0), m), k, _ptr(U),
                              _ptr(S), _ptr(V), _ptr(info), _ptr(ws), ws.numel(),
                              _stream_ptr(stream)))
    return U, S, V, info


def bsrht_dense_workspace(n, l, m):
    return int(lib().bsrht_dense_workspace(n, l, m))


def bsrht_dense_sketch(kind, seed, l, A, Y=None, ws=None, stream=None):
    """Y = G A for a dense Gaussian (DENSE_GAUSSIAN) or Rademacher
    (DENSE_RADEMACHER) l x n G drawn from (seed); A: n x m float32."""
    _check_matrix("A", A)
    n, m = A.shape
    if Y is None:
        Y = torch.empty(l, m, dtype=torch.float32, device=A.device)
    _check_matrix("Y", Y)
    if tuple(Y.shape) != (l, m):
        raise ValueError(f"Y must be {l} x {m}")
    if ws is None:
        ws = _workspace(bsrht_dense_workspace(n, l, m), A.device)
    _check("bsrht_dense_sketch", lib().bsrht_dense_sketch(
        kind, ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), n, l, _ptr(A), m, max(A.stride(0), m),
        _ptr(Y), max(Y.stride(0), m), _ptr(ws), ws.numel(), _stream_ptr(stream)))
    return Y


def rsvd_single_view_workspace(omega, gamma, phi, psi, k):
    return int(lib().rsvd_single_view_workspace(omega.handle, gamma.handle, phi.handle,
                                                psi.handle, k))


def _single_view_args(omega, gamma, phi, psi, A, k, ws):
    _check_matrix("A", A)
    N1, N2 = A.shape
    if N1 != gamma.n or N2 != omega.n:
        raise ValueError(f"A is {N1} x {N2}; the plans expect {gamma.n} x {omega.n}")
    dev = A.device
    U = torch.empty(N1, k, dtype=torch.float32, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty(N2, k, dtype=torch.float32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if ws is None:
        need = rsvd_single_view_workspace(omega, gamma, phi, psi, k)
        if need == 0:
            raise ValueError("inconsistent single-view plans")
        ws = _workspace(need, dev)
    args = (omega.handle, gamma.handle, phi.handle, psi.handle, _ptr(A), max(A.stride(0), N2), k,
            _ptr(U), _ptr(S), _ptr(V), _ptr(info), _ptr(ws), ws.numel())
    return args, U, S, V, info, ws


def rsvd_single_view(omega, gamma, phi, psi, A, k, ws=None, stream=None):
    """Single-view RSVD (Algorithm 3) of the N1 x N2 A with Omega (l x N2),
    Gamma (l x N1), Phi (s x N1), Psi (s x N2): returns (U N1 x k, S k
    float64, V N2 x k, info), A ~= U diag(S) V^T."""
    args, U, S, V, info, _ = _single_view_args(omega, gamma, phi, psi, A, k, ws)
    _check("rsvd_single_view", lib().rsvd_single_view(*args, _stream_ptr(stream)))
    return U, S, V, info


def rsvd_single_view_start(omega, gamma, phi, psi, A, k, ws=None, stream=None):
    """Non-blocking rsvd_single_view: returns (task, U, S, V, info), valid as
    for rsvd_start."""
    args, U, S, V, info, ws = _single_view_args(omega, gamma, phi, psi, A, k, ws)
    h = _c_vp()
    _check("rsvd_single_view_start",
           lib().rsvd_single_view_start(*args, _stream_ptr(stream), ctypes.byref(h)))
    return Task(h.value, (omega, gamma, phi, psi, A, U, S, V, info, ws)), U, S, V, info


def nystrom_workspace(plan, k):
    return int(lib().nystrom_workspace(plan.handle, k))


def nystrom(plan, A, k, ws=None, stream=None, shifted=False):
    """Nystrom (Algorithm 2) of symmetric PSD A: returns (U n x k, lambda k float64, info).
    shifted=True runs it on A + nu I and subtracts nu (nystrom_shifted)."""
    _check_matrix("A", A)
    n = A.shape[0]
    if A.shape[1] != n or n != plan.n:
        raise ValueError("A must be n x n with n = plan.n")
    dev = A.device
    U = torch.empty(n, k, dtype=torch.float32, device=dev)
    lam = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = _workspace(nystrom_workspace(plan, k), dev)
    name = "nystrom_shifted" if shifted else "nystrom"
    _check(name, getattr(lib(), name)(plan.handle, _ptr(A), max(A.stride(0), n), k, _ptr(U),
                                      _ptr(lam), _ptr(info), _ptr(ws), ws.numel(),
                                      _stream_ptr(stream)))
    return U, lam, info


def nystrom_shifted(plan, A, k, ws=None, stream=None):
    """Shifted Nystrom (on A + nu I, nu subtracted): returns (U, lambda, info)."""
    return nystrom(plan, A, k, ws, stream, shifted=True)


class Task:
    """A non-blocking rsvd / nystrom / single-view call (rsvd_start,
    nystrom_start, rsvd_single_view_start of include/bsrht.h).  poll() advances it without waiting and returns True once
    all of its work is queued (raising if the call failed); wait() blocks until
    then.  The results are ready in stream order.  The tensors the call uses
    are kept alive until the task is closed."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def poll(self):
        st = ctypes.c_int(0)
        r = lib().bsrht_task_poll(self.handle, ctypes.byref(st))
        if r < 0:
            _check("bsrht_task_poll", r)
        if r == 1:
            _check("task", st.value)
            return True
        return False

    def wait(self):
        _check("bsrht_task_wait", lib().bsrht_task_wait(self.handle))

    def close(self):
        h, self.handle = self.handle, None
        if h is not None and _lib is not None:
            _check("bsrht_task_destroy", _lib.bsrht_task_destroy(h))
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rsvd_start(plan, A, k, ws=None, stream=None):
    """Non-blocking rsvd: returns (task, U, S, V, info); the outputs are
    valid once task.poll() returned True (or task.wait()) and the stream has
    reached the task's end."""
    _check_matrix("A", A)
    n, m = A.shape
    if n != plan.n:
        raise ValueError(f"A has {n} rows, the plan expects {plan.n}")
    dev = A.device
    U = torch.empty(n, k, dtype=torch.float32, device=dev)
    S = torch.empty(k, dtype=torch.float64, device=dev)
    V = torch.empty(m, k, dtype=torch.float32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = _workspace(rsvd_workspace(plan, m, k), dev)
    h = _c_vp()
    _check("rsvd_start", lib().rsvd_start(plan.handle, _ptr(A), m, max(A.stride(0), m), k,
                                          _ptr(U), _ptr(S), _ptr(V), _ptr(info), _ptr(ws),
                                          ws.numel(), _stream_ptr(stream), ctypes.byref(h)))
    return Task(h.value, (plan, A, U, S, V, info, ws)), U, S, V, info


def nystrom_start(plan, A, k, ws=None, stream=None, shifted=False):
    """Non-blocking nystrom (nystrom_shifted with shifted=True): returns
    (task, U, lambda, info), valid as for rsvd_start."""
    _check_matrix("A", A)
    n = A.shape[0]
    if A.shape[1] != n or n != plan.n:
        raise ValueError("A must be n x n with n = plan.n")
    dev = A.device
    U = torch.empty(n, k, dtype=torch.float32, device=dev)
    lam = torch.empty(k, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = _workspace(nystrom_workspace(plan, k), dev)
    name = "nystrom_shifted_start" if shifted else "nystrom_start"
    h = _c_vp()
    _check(name, getattr(lib(), name)(plan.handle, _ptr(A), max(A.stride(0), n), k, _ptr(U),
                                      _ptr(lam), _ptr(info), _ptr(ws), ws.numel(),
                                      _stream_ptr(stream), ctypes.byref(h)))
    return Task(h.value, (plan, A, U, lam, info, ws)), U, lam, info


def bsrht_job_bytes(job):
    """Arena bytes a JobDesc needs on a plan-cache miss (0 if invalid)."""
    return int(lib().bsrht_job_bytes(ctypes.byref(job)))


class Server:
    """The serving runtime of include/bsrht_serve.h.

    Server(arena=tensor, workers=W) runs up to W jobs at a time on the GPU,
    one per stream slot, inside the uint8 device tensor `arena` (the HBM
    budget); jobs advance while submit / poll / drain are called.
    Server(fake_bytes=B, workers=W, seconds_per_gb=t) is the host-only
    executor with a B-byte budget.  Device pointers of submitted jobs must
    stay alive until their result has been polled; the caller keeps the
    tensors.
    """

    def __init__(self, arena=None, workers=4, fake_bytes=None, seconds_per_gb=0.0):
        L = lib()
        h = ctypes.c_void_p()
        if fake_bytes is not None:
            st = L.bsrht_server_create_fake(int(fake_bytes), int(workers),
                                            float(seconds_per_gb), ctypes.byref(h))
            self.arena = None
        else:
            if not isinstance(arena, torch.Tensor) or not arena.is_cuda:
                raise ValueError("arena must be a device tensor")
            self.arena = arena
            with torch.cuda.device(arena.device):
                st = L.bsrht_server_create(_ptr(arena), arena.numel() * arena.element_size(),
                                           int(workers), ctypes.byref(h))
        _check("bsrht_server_create", st)
        self.handle = h

    def submit(self, job):
        st = lib().bsrht_server_submit(self.handle, ctypes.byref(job))
        _check("bsrht_server_submit", st)

    def submit_many(self, jobs):
        """Submits a list of JobDesc at once; returns how many were accepted
        (raises on the first rejected one after submitting those before it)."""
        arr = (JobDesc * max(len(jobs), 1))(*jobs)
        acc = ctypes.c_int()
        st = lib().bsrht_server_submit_many(self.handle, arr, len(jobs), ctypes.byref(acc))
        _check("bsrht_server_submit_many", st)
        return acc.value

    def poll(self, max_results=256, timeout=0.0):
        buf = (JobResult * max_results)()
        c = ctypes.c_int()
        _check("bsrht_server_poll", lib().bsrht_server_poll(self.handle, buf, max_results,
                                                            float(timeout), ctypes.byref(c)))
        return [buf[i] for i in range(c.value)]

    def drain(self):
        _check("bsrht_server_drain", lib().bsrht_server_drain(self.handle))

    def stats(self):
        out = ServerStats()
        _check("bsrht_server_stats", lib().bsrht_server_stats(self.handle, ctypes.byref(out)))
        return {name: getattr(out, name) for name, _ in ServerStats._fields_}

    def set_batching(self, on):
        _check("bsrht_server_set_batching", lib().bsrht_server_set_batching(self.handle, int(on)))

    def clock(self):
        return float(lib().bsrht_server_clock(self.handle))

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _check("bsrht_server_destroy", _lib.bsrht_server_destroy(h))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def sketch_job(job_id, plan_args, A, Y):
    """JobDesc for Y = Omega A; plan_args = (n, p, l, seed, sampling, precision)."""
    n, p, l, seed, sampling, precision = plan_args
    _check_matrix("A", A)
    _check_matrix("Y", Y)
    m = A.shape[1]
    return JobDesc(id=job_id, kind=JOB_SKETCH, n=n, m=m, p=p, l=l, k=0,
                   seed=int(seed) & (2 ** 64 - 1), sampling=sampling, precision=precision,
                   A=A.data_ptr(), lda=max(A.stride(0), m), Y=Y.data_ptr(),
                   ldy=max(Y.stride(0), m))


def nystrom_job(job_id, plan_args, A, k, U, lam, info):
    """JobDesc for the Nystrom approximation of the symmetric PSD n x n A into
    caller-owned U (n x k), lam (k, float64) and info."""
    n, p, l, seed, sampling, precision = plan_args
    _check_matrix("A", A)
    if A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    m = A.shape[1]
    return JobDesc(id=job_id, kind=JOB_NYSTROM, n=n, m=m, p=p, l=l, k=k,
                   seed=int(seed) & (2 ** 64 - 1), sampling=sampling, precision=precision,
                   A=A.data_ptr(), lda=max(A.stride(0), m), U=U.data_ptr(), S=lam.data_ptr(),
                   info=info.data_ptr())


def finalize():
    """bsrht_finalize: release the library's process-lifetime HIP objects now
    (also done automatically at interpreter exit)."""
    _check("bsrht_finalize", lib().bsrht_finalize())


def rsvd_job(job_id, plan_args, A, k, U, S, V, info):
    """JobDesc for the randomized SVD of A into caller-owned U, S, V, info."""
    n, p, l, seed, sampling, precision = plan_args
    _check_matrix("A", A)
    m = A.shape[1]
    return JobDesc(id=job_id, kind=JOB_RSVD, n=n, m=m, p=p, l=l, k=k,
                   seed=int(seed) & (2 ** 64 - 1), sampling=sampling, precision=precision,
                   A=A.data_ptr(), lda=max(A.stride(0), m), U=U.data_ptr(), S=S.data_ptr(),
                   V=V.data_ptr(), info=info.data_ptr())
