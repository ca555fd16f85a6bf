"""MI355X (gfx950) alpha-dense DFT -- Python binding of the C ABI in include/dense_dft.h.

The transform (paper Section 2, eq. (7) on the grid of eq. (6), T/N factor of
eq. (2)):  X_m = (T/N) sum_{n<N} x_n exp(-2 pi i m n / (alpha N)),
m < alpha N, computed on the GPU in the FFT-structured form of Section 3.

This module only marshals arguments: it passes device pointers taken from
torch tensors and the current HIP stream to ``libdensedft.so``; every step of
the transform runs in the library's HIP kernels.  Importing it fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdensedft.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)

DD_F32, DD_C64, DD_F64, DD_C128 = 0, 1, 2, 3
DD_TWIDDLE_FP64, DD_TWIDDLE_FP32 = 0, 1
DD_NO_WORKSPACE = 2
DD_SERVE_BATCHED, DD_SERVE_PLAIN = 0, 1
DD_SERVE_DETERMINISTIC = 0x100
STATUS = {0: "DD_OK", 1: "DD_ERR_INVALID", 2: "DD_ERR_UNSUPPORTED", 3: "DD_ERR_NOMEM",
          4: "DD_ERR_DEVICE", 5: "DD_ERR_BUSY", 6: "DD_ERR_TOO_LARGE", 7: "DD_ERR_TIMEOUT",
          8: "DD_ERR_CLOSED"}

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_lib.dense_dft_plan.argtypes = [ctypes.POINTER(_vp), _i64, ctypes.c_int32, ctypes.c_double, _i64,
                                ctypes.c_int, ctypes.c_uint32]
_lib.dense_dft_plan.restype = ctypes.c_int
_lib.dense_dft_exec.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.dense_dft_exec.restype = ctypes.c_int
_lib.dense_dft_plan_decimated.argtypes = [ctypes.POINTER(_vp), _i64, ctypes.c_int32, ctypes.c_double, _i64,
                                          ctypes.c_int, ctypes.c_uint32]
_lib.dense_dft_plan_decimated.restype = ctypes.c_int
_lib.dense_dft_exec_static.argtypes = [_vp, _vp, _vp, _vp]
_lib.dense_dft_exec_static.restype = ctypes.c_int
_lib.dense_dft_exec_inverse.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.dense_dft_exec_inverse.restype = ctypes.c_int
_lib.dense_dft_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.dense_dft_workspace_size.restype = ctypes.c_int
_lib.dense_dft_destroy.argtypes = [_vp]
_lib.dense_dft_destroy.restype = ctypes.c_int
_lib.dense_dft_plan_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_i64),
                                     ctypes.POINTER(_i64)]
_lib.dense_dft_plan_info.restype = ctypes.c_int
_lib.dense_dft_profile_begin.argtypes = [_vp, ctypes.c_int32]
_lib.dense_dft_profile_begin.restype = ctypes.c_int
_lib.dense_dft_profile_end.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
_lib.dense_dft_profile_end.restype = ctypes.c_int


class dd_sched(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("lines", ctypes.c_int32), ("N1", ctypes.c_int64),
                ("N2", ctypes.c_int64), ("jgroup", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("chunk", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


class dd_tune_info(ctypes.Structure):
    _fields_ = [("best", dd_sched), ("ms_best", ctypes.c_float), ("ms_default", ctypes.c_float),
                ("candidates", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib.dense_dft_plan_sched.argtypes = [ctypes.POINTER(_vp), _i64, ctypes.c_int32, ctypes.c_double, _i64,
                                      ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(dd_sched)]
_lib.dense_dft_plan_sched.restype = ctypes.c_int
_lib.dense_dft_plan_get_sched.argtypes = [_vp, ctypes.POINTER(dd_sched)]
_lib.dense_dft_plan_get_sched.restype = ctypes.c_int
_lib.dense_dft_sched_candidates.argtypes = [_i64, ctypes.c_int32, _i64, ctypes.c_int, ctypes.POINTER(dd_sched),
                                            ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
_lib.dense_dft_sched_candidates.restype = ctypes.c_int
_lib.dense_dft_batch_sched_candidates.argtypes = [_i64, ctypes.c_int32, ctypes.POINTER(dd_sched), ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_int32)]
_lib.dense_dft_batch_sched_candidates.restype = ctypes.c_int
_lib.dense_dft_tune.argtypes = [_i64, ctypes.c_int32, _i64, ctypes.c_int, ctypes.POINTER(dd_tune_info)]
_lib.dense_dft_tune.restype = ctypes.c_int
_lib.dense_dft_tune_batch.argtypes = [_i64, ctypes.c_int32, ctypes.POINTER(dd_tune_info)]
_lib.dense_dft_tune_batch.restype = ctypes.c_int
_lib.dense_dft_tune_save.argtypes = [ctypes.c_char_p]
_lib.dense_dft_tune_save.restype = ctypes.c_int
_lib.dense_dft_tune_load.argtypes = [ctypes.c_char_p]
_lib.dense_dft_tune_load.restype = ctypes.c_int
_lib.dense_dft_tune_clear.argtypes = []
_lib.dense_dft_tune_clear.restype = ctypes.c_int
_lib.dense_dft_tune_entries.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
_lib.dense_dft_tune_entries.restype = ctypes.c_int


class dd_desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("alpha", ctypes.c_int32), ("T", ctypes.c_double),
                ("dtype", ctypes.c_int), ("x", ctypes.c_void_p), ("X", ctypes.c_void_p)]


_lib.dense_dft_batch_plan.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(dd_desc), ctypes.c_int32,
                                      ctypes.c_uint32]
_lib.dense_dft_batch_plan.restype = ctypes.c_int
_lib.dense_dft_batch_plan_sched.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(dd_desc), ctypes.c_int32,
                                            ctypes.c_uint32, ctypes.POINTER(dd_sched)]
_lib.dense_dft_batch_plan_sched.restype = ctypes.c_int
_lib.dense_dft_batch_exec.argtypes = [_vp, _vp]
_lib.dense_dft_batch_exec.restype = ctypes.c_int
_lib.dense_dft_batch_set_buffers.argtypes = [_vp, ctypes.POINTER(dd_desc), ctypes.c_int32]
_lib.dense_dft_batch_set_buffers.restype = ctypes.c_int
_lib.dense_dft_batch_status.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint32)]
_lib.dense_dft_batch_status.restype = ctypes.c_int
_lib.dense_dft_batch_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32)]
_lib.dense_dft_batch_info.restype = ctypes.c_int
_lib.dense_dft_batch_destroy.argtypes = [_vp]
_lib.dense_dft_batch_destroy.restype = ctypes.c_int
_lib.dense_dft_exec_many.argtypes = [ctypes.POINTER(dd_desc), ctypes.c_int32, _vp]
_lib.dense_dft_exec_many.restype = ctypes.c_int
_lib.dense_dft_status_string.argtypes = [ctypes.c_int]
_lib.dense_dft_status_string.restype = ctypes.c_char_p
_lib.dense_dft_version.argtypes = []
_lib.dense_dft_version.restype = ctypes.c_int32


class DenseDFTError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} "
                         f"({_lib.dense_dft_status_string(status).decode()})")


def _check(rc: int, what: str):
    if rc != 0:
        raise DenseDFTError(rc, what)


def dense_dft_status_string(status: int) -> str:
    return _lib.dense_dft_status_string(int(status)).decode()


def dense_dft_version() -> int:
    return int(_lib.dense_dft_version())


class Plan:
    """Owning handle of a dd_plan_t; destroyed when garbage-collected."""

    _destroy = _lib.dense_dft_destroy  # kept on the class: usable at interpreter exit

    def __init__(self, handle, N, alpha, T, batch, dtype, flags):
        self.handle = handle
        self.N, self.alpha, self.T, self.batch = N, alpha, T, batch
        self.dtype, self.flags = dtype, flags

    @property
    def M(self) -> int:
        """Bins per signal: alpha*N, or N/p for an alpha = 1/p plan."""
        p = getattr(self, "p", 0)
        return self.N // p if p else self.alpha * self.N

    def exec(self, x, out=None, stream=None, workspace=None):
        """Enqueue the transform of device tensor x ([batch, N] of the plan's
        dtype) into ``out`` ([batch, M] complex; allocated when None) on
        ``stream`` (default: torch's current stream); returns ``out``."""
        if out is None:
            import torch
            out = torch.empty((self.batch, self.M), dtype=out_dtype(self.dtype), device=x.device)
        dense_dft_exec(self, x, out, workspace, stream)
        return out

    def exec_inverse(self, X, out=None, stream=None, workspace=None):
        """Enqueue the inverse transform of device spectra X ([batch, alpha*N])
        into ``out`` ([batch, N] complex; allocated when None); returns ``out``."""
        if out is None:
            import torch
            out = torch.empty((self.batch, self.N), dtype=out_dtype(self.dtype), device=X.device)
        dense_dft_exec_inverse(self, X, out, workspace, stream)
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._destroy(h)
            self.handle = None


def dense_dft_plan(N: int, alpha: int, T: float, batch: int, dtype: int,
                   flags: int = DD_TWIDDLE_FP64) -> Plan:
    h = _vp()
    _check(_lib.dense_dft_plan(ctypes.byref(h), int(N), int(alpha), float(T), int(batch),
                               int(dtype), int(flags)), "dense_dft_plan")
    return Plan(h, int(N), int(alpha), float(T), int(batch), int(dtype), int(flags))


def plan(N: int, alpha: int, T: float, batch: int, dtype, flags: int = DD_TWIDDLE_FP64) -> Plan:
    """dense_dft_plan with ``dtype`` a DD_* code or a torch dtype
    (float32, complex64, float64, complex128)."""
    code = dtype if isinstance(dtype, int) else dtype_code(dtype)
    return dense_dft_plan(N, alpha, T, batch, code, flags)


def dense_dft_workspace_size(plan: Plan) -> int:
    n = ctypes.c_size_t()
    _check(_lib.dense_dft_workspace_size(plan.handle, ctypes.byref(n)), "dense_dft_workspace_size")
    return int(n.value)


def dense_dft_plan_info(plan: Plan):
    """(passes, N1, N2) of the schedule the plan chose."""
    p, n1, n2 = ctypes.c_int32(), _i64(), _i64()
    _check(_lib.dense_dft_plan_info(plan.handle, ctypes.byref(p), ctypes.byref(n1),
                                    ctypes.byref(n2)), "dense_dft_plan_info")
    return int(p.value), int(n1.value), int(n2.value)


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def in_dtype(code: int):
    """torch dtype of a DD_* input code."""
    import torch
    return {DD_F32: torch.float32, DD_C64: torch.complex64, DD_F64: torch.float64,
            DD_C128: torch.complex128}[code]


def _check_buf(t, what: str, dtype, numel: int) -> None:
    """The C ABI sees only an address, so a tensor the kernels will read or
    write is checked here: on the device, of the plan's dtype, contiguous,
    and holding at least the ``numel`` elements the launch touches.  Raises
    DenseDFTError with DD_ERR_INVALID, as the library does for bad arguments."""
    if not getattr(t, "is_cuda", False):
        where = f" on {t.device}" if hasattr(t, "device") else ""
        raise DenseDFTError(1, f"{what}: expected a device (cuda) tensor, got {type(t).__name__}{where}")
    if t.dtype != dtype:
        raise DenseDFTError(1, f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise DenseDFTError(1, f"{what}: the tensor must be contiguous")
    if t.numel() < numel:
        raise DenseDFTError(1, f"{what}: {t.numel()} elements, the transform needs {numel}")


def _check_workspace(plan, workspace) -> None:
    if workspace is None:
        return
    if not getattr(workspace, "is_cuda", False) or not workspace.is_contiguous():
        raise DenseDFTError(1, "workspace: expected a contiguous device (cuda) tensor")
    have, need = workspace.numel() * workspace.element_size(), dense_dft_workspace_size(plan)
    if have < need:
        raise DenseDFTError(1, f"workspace: {have} bytes, the plan needs {need}")


def dense_dft_exec(plan: Plan, x, X, workspace=None, stream=None) -> None:
    """Enqueue the plan on ``stream`` (default: torch's current stream).

    x: device tensor [batch, N] of the plan's dtype; X: device complex tensor
    [batch, alpha*N]; workspace: optional device tensor of at least
    dense_dft_workspace_size(plan) bytes.
    """
    _check_buf(x, "x", in_dtype(plan.dtype), plan.batch * plan.N)
    _check_buf(X, "X", out_dtype(plan.dtype), plan.batch * plan.M)
    _check_workspace(plan, workspace)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(x.device).cuda_stream
    _check(_lib.dense_dft_exec(plan.handle, _ptr(x), _ptr(X), _ptr(workspace), _vp(stream)),
           "dense_dft_exec")


DD_STATIC_SCRATCH_BYTES = 64 << 20


def dense_dft_exec_static(plan: Plan, x, X, stream=None) -> None:
    """The forward transform without any allocation: the two-pass scratch is
    the library's fixed per-device array of DD_STATIC_SCRATCH_BYTES (calls on
    one device share it, so their executions must not overlap in time).
    x, X, stream: as dense_dft_exec."""
    _check_buf(x, "x", in_dtype(plan.dtype), plan.batch * plan.N)
    _check_buf(X, "X", out_dtype(plan.dtype), plan.batch * plan.M)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(x.device).cuda_stream
    _check(_lib.dense_dft_exec_static(plan.handle, _ptr(x), _ptr(X), _vp(stream)), "dense_dft_exec_static")


KERNEL_KINDS = {1: "single", 2: "pass1", 3: "pass2", 4: "inverse_single", 5: "inverse_passA", 6: "inverse_passB"}


def dense_dft_profile_begin(plan: Plan, max_launches: int) -> None:
    _check(_lib.dense_dft_profile_begin(plan.handle, int(max_launches)), "dense_dft_profile_begin")


def dense_dft_profile_end(plan: Plan, cap: int = 4096):
    """List of (kind, milliseconds) for each launch recorded since profile_begin."""
    kinds = (ctypes.c_int32 * cap)()
    ms = (ctypes.c_float * cap)()
    n = ctypes.c_int32()
    _check(_lib.dense_dft_profile_end(plan.handle, kinds, ms, int(cap), ctypes.byref(n)),
           "dense_dft_profile_end")
    return [(KERNEL_KINDS.get(kinds[i], str(kinds[i])), float(ms[i])) for i in range(n.value)]


def dense_dft_destroy(plan: Plan) -> None:
    if plan.handle:
        _check(_lib.dense_dft_destroy(plan.handle), "dense_dft_destroy")
        plan.handle = None


# --- schedules and the tuner ---
def make_sched(passes: int, N1: int = 0, N2: int = 0, jgroup: int = 0, lines: int = 0, chunk: int = 0) -> dd_sched:
    return dd_sched(int(passes), int(lines), int(N1), int(N2), int(jgroup), 0, int(chunk))


def dense_dft_plan_sched(N: int, alpha: int, T: float, batch: int, dtype: int, sched: dd_sched,
                         flags: int = DD_TWIDDLE_FP64) -> Plan:
    h = _vp()
    _check(_lib.dense_dft_plan_sched(ctypes.byref(h), int(N), int(alpha), float(T), int(batch), int(dtype),
                                     int(flags), ctypes.byref(sched)), "dense_dft_plan_sched")
    return Plan(h, N, alpha, T, batch, dtype, flags)


def dense_dft_plan_get_sched(plan: Plan) -> dict:
    sc = dd_sched()
    _check(_lib.dense_dft_plan_get_sched(plan.handle, ctypes.byref(sc)), "dense_dft_plan_get_sched")
    return sc.as_dict()


def dense_dft_sched_candidates(N: int, alpha: int, batch: int, dtype: int) -> list:
    n = ctypes.c_int32()
    _check(_lib.dense_dft_sched_candidates(int(N), int(alpha), int(batch), int(dtype), None, 0, ctypes.byref(n)),
           "dense_dft_sched_candidates")
    arr = (dd_sched * n.value)()
    _check(_lib.dense_dft_sched_candidates(int(N), int(alpha), int(batch), int(dtype), arr, n.value,
                                           ctypes.byref(n)), "dense_dft_sched_candidates")
    return list(arr)


def dense_dft_batch_sched_candidates(N: int, alpha: int) -> list:
    n = ctypes.c_int32()
    arr = (dd_sched * 16)()
    _check(_lib.dense_dft_batch_sched_candidates(int(N), int(alpha), arr, 16, ctypes.byref(n)),
           "dense_dft_batch_sched_candidates")
    return list(arr)[:n.value]


def _tune_dict(info: dd_tune_info) -> dict:
    return {"best": info.best.as_dict(), "ms_best": float(info.ms_best), "ms_default": float(info.ms_default),
            "candidates": int(info.candidates)}


def dense_dft_tune(N: int, alpha: int, batch: int, dtype: int) -> dict:
    info = dd_tune_info()
    _check(_lib.dense_dft_tune(int(N), int(alpha), int(batch), int(dtype), ctypes.byref(info)), "dense_dft_tune")
    return _tune_dict(info)


def dense_dft_tune_batch(N: int, alpha: int) -> dict:
    info = dd_tune_info()
    _check(_lib.dense_dft_tune_batch(int(N), int(alpha), ctypes.byref(info)), "dense_dft_tune_batch")
    return _tune_dict(info)


def dense_dft_tune_save(path: str) -> None:
    _check(_lib.dense_dft_tune_save(os.fsencode(path)), "dense_dft_tune_save")


def dense_dft_tune_load(path: str) -> None:
    _check(_lib.dense_dft_tune_load(os.fsencode(path)), "dense_dft_tune_load")


def dense_dft_tune_clear() -> None:
    _check(_lib.dense_dft_tune_clear(), "dense_dft_tune_clear")


def dense_dft_tune_entries():
    """(plain-plan entries, batch-kernel class entries) of the tuning table."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.dense_dft_tune_entries(ctypes.byref(a), ctypes.byref(b)), "dense_dft_tune_entries")
    return int(a.value), int(b.value)


# --- many signals of uneven N and alpha in one persistent launch ---
class Batch:
    """Owning handle of a dd_batch_t.  It keeps the tensors its descriptors
    name, so that they outlive every execution the plan may still make."""

    _destroy = _lib.dense_dft_batch_destroy

    def __init__(self, handle, count, tensors=()):
        self.handle = handle
        self.count = count
        self.tensors = list(tensors)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._destroy(h)
            self.handle = None


def _desc_tensors(descs):
    """The tensors named by (N, alpha, T, dtype, x, X) descriptors."""
    out = []
    for d in descs:
        if not isinstance(d, dd_desc):
            out += [t for t in d[4:6] if t is not None]
    return out


def _desc_array(descs):
    """descs: iterable of (N, alpha, T, dtype, x_tensor, X_tensor) or dd_desc."""
    items = list(descs)
    arr = (dd_desc * len(items))()
    for i, d in enumerate(items):
        if isinstance(d, dd_desc):
            arr[i] = d
        else:
            arr[i] = _one_desc(d, f"descriptor {i}")
    return arr, len(items)


def dense_dft_batch_plan(descs, flags: int = DD_TWIDDLE_FP64) -> Batch:
    """Plan one persistent launch over the descriptors (N, alpha, T, dtype, x, X).
    The returned Batch keeps x and X alive (a dd_desc passes raw addresses, and
    its buffers are the caller's to keep)."""
    descs = list(descs)
    arr, n = _desc_array(descs)
    h = _vp()
    _check(_lib.dense_dft_batch_plan(ctypes.byref(h), arr, n, int(flags)), "dense_dft_batch_plan")
    return Batch(h, n, _desc_tensors(descs))


def dense_dft_batch_plan_sched(descs, sched: dd_sched, flags: int = DD_TWIDDLE_FP64) -> Batch:
    descs = list(descs)
    arr, n = _desc_array(descs)
    h = _vp()
    _check(_lib.dense_dft_batch_plan_sched(ctypes.byref(h), arr, n, int(flags), ctypes.byref(sched)),
           "dense_dft_batch_plan_sched")
    return Batch(h, n, _desc_tensors(descs))


def dense_dft_batch_exec(batch: Batch, stream=None) -> None:
    """Enqueue the batch on ``stream`` (default: torch's current stream); the
    inputs must have been written by work ordered before it on that stream."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.dense_dft_batch_exec(batch.handle, _vp(stream)), "dense_dft_batch_exec")


def dense_dft_batch_set_buffers(batch: Batch, descs) -> None:
    """New buffers for the next executions (same shapes); the batch then keeps
    the new tensors instead of the old ones.  Executions already enqueued
    still use the old buffers: synchronise their stream before freeing those."""
    descs = list(descs)
    arr, n = _desc_array(descs)
    _check(_lib.dense_dft_batch_set_buffers(batch.handle, arr, n), "dense_dft_batch_set_buffers")
    batch.tensors = _desc_tensors(descs)


def dense_dft_batch_status(batch: Batch) -> int:
    f = ctypes.c_uint32()
    _check(_lib.dense_dft_batch_status(batch.handle, ctypes.byref(f)), "dense_dft_batch_status")
    return int(f.value)


def dense_dft_batch_info(batch: Batch):
    """(tasks, grid, scratch_bytes, fallback_signals)."""
    t, g, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    sb = ctypes.c_size_t()
    _check(_lib.dense_dft_batch_info(batch.handle, ctypes.byref(t), ctypes.byref(g), ctypes.byref(sb),
                                     ctypes.byref(f)), "dense_dft_batch_info")
    return int(t.value), int(g.value), int(sb.value), int(f.value)


def dense_dft_batch_destroy(batch: Batch) -> None:
    if batch.handle:
        _check(_lib.dense_dft_batch_destroy(batch.handle), "dense_dft_batch_destroy")
        batch.handle = None


def dense_dft_exec_many(descs, stream=None) -> None:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    arr, n = _desc_array(descs)
    _check(_lib.dense_dft_exec_many(arr, n, _vp(stream)), "dense_dft_exec_many")


# --- serving: continuous batching of requests as they arrive ---
class dd_server_cfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("mode", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t),
                ("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p), ("batch_max_bins", ctypes.c_int64),
                ("spin_us", ctypes.c_int32)]


class dd_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("batch_requests", ctypes.c_int32), ("t_arrival_ns", ctypes.c_uint64),
                ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class dd_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("kernel_requests", ctypes.c_uint64), ("fallback_requests", ctypes.c_uint64),
                ("max_batch_seen", ctypes.c_int32), ("classes", ctypes.c_int32), ("pool_bytes", ctypes.c_size_t),
                ("peak_footprint", ctypes.c_size_t)]


_u64 = ctypes.c_uint64
_lib.dense_dft_server_create.argtypes = [ctypes.POINTER(dd_server_cfg), ctypes.POINTER(_vp)]
_lib.dense_dft_server_create.restype = ctypes.c_int
_lib.dense_dft_server_warm.argtypes = [_vp, _i64, ctypes.c_int32, ctypes.c_double, ctypes.c_int]
_lib.dense_dft_server_warm.restype = ctypes.c_int
_lib.dense_dft_submit.argtypes = [_vp, ctypes.POINTER(dd_desc), ctypes.POINTER(_u64)]
_lib.dense_dft_submit.restype = ctypes.c_int
_lib.dense_dft_submit_at.argtypes = [_vp, ctypes.POINTER(dd_desc), _u64, ctypes.POINTER(_u64)]
_lib.dense_dft_submit_at.restype = ctypes.c_int
_lib.dense_dft_submit_many_at.argtypes = [_vp, ctypes.POINTER(dd_desc), ctypes.POINTER(_u64), ctypes.c_int32,
                                          ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_int32)]
_lib.dense_dft_submit_many_at.restype = ctypes.c_int
_lib.dense_dft_poll.argtypes = [_vp, _u64, ctypes.POINTER(dd_result)]
_lib.dense_dft_poll.restype = ctypes.c_int
_lib.dense_dft_wait.argtypes = [_vp, _u64, _i64, ctypes.POINTER(dd_result)]
_lib.dense_dft_wait.restype = ctypes.c_int
_lib.dense_dft_server_pause.argtypes = [_vp, ctypes.c_int32]
_lib.dense_dft_server_pause.restype = ctypes.c_int
_lib.dense_dft_server_stats.argtypes = [_vp, ctypes.POINTER(dd_server_stats)]
_lib.dense_dft_server_stats.restype = ctypes.c_int
_lib.dense_dft_server_destroy.argtypes = [_vp]
_lib.dense_dft_server_destroy.restype = ctypes.c_int
_lib.dense_dft_clock_ns.argtypes = []
_lib.dense_dft_clock_ns.restype = _u64

DD_ERR_BUSY, DD_ERR_TOO_LARGE, DD_ERR_TIMEOUT, DD_ERR_CLOSED = 5, 6, 7, 8


class Server:
    """Owning handle of a dd_server_t (destroyed, after draining, when collected)."""

    _destroy = _lib.dense_dft_server_destroy

    def __init__(self, handle, cfg):
        self.handle = handle
        self.cfg = cfg
        self.pending = {}   # ticket -> the tensors of its request, until its result is taken

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._destroy(h)
            self.handle = None


def dense_dft_server_create(device: int = 0, mode: int = DD_SERVE_BATCHED, hbm_budget_bytes: int = 0,
                            max_inflight: int = 0, max_batch: int = 0, max_queue: int = 0,
                            flags: int = DD_TWIDDLE_FP64, hip_stream=None, batch_max_bins: int = 0,
                            spin_us: int = 0) -> Server:
    cfg = dd_server_cfg(int(device), int(mode), int(hbm_budget_bytes), int(max_inflight), int(max_batch),
                        int(max_queue), int(flags), hip_stream, int(batch_max_bins), int(spin_us))
    h = _vp()
    _check(_lib.dense_dft_server_create(ctypes.byref(cfg), ctypes.byref(h)), "dense_dft_server_create")
    return Server(h, cfg)


def dense_dft_server_warm(server: Server, N: int, alpha: int, T: float, dtype: int) -> None:
    _check(_lib.dense_dft_server_warm(server.handle, int(N), int(alpha), float(T), int(dtype)),
           "dense_dft_server_warm")


def _one_desc(d, what: str = "request") -> dd_desc:
    """dd_desc from (N, alpha, T, dtype, x_tensor, X_tensor); the tensors are
    checked against N, alpha and dtype (None passes as NULL, which the library
    refuses).  A dd_desc passes through unchecked."""
    if isinstance(d, dd_desc):
        return d
    N, alpha, T, dtype, x, X = d
    if dtype in (DD_F32, DD_C64, DD_F64, DD_C128) and int(N) > 0 and int(alpha) > 0:
        if x is not None:
            _check_buf(x, f"{what}: x", in_dtype(dtype), int(N))
        if X is not None:
            _check_buf(X, f"{what}: X", out_dtype(dtype), int(alpha) * int(N))
    return dd_desc(int(N), int(alpha), float(T), int(dtype), None if x is None else x.data_ptr(),
                   None if X is None else X.data_ptr())


def dense_dft_submit(server: Server, desc, t_arrival_ns: int | None = None) -> int:
    """Queue one request (N, alpha, T, dtype, x_tensor, X_tensor); returns its ticket.
    Raises DenseDFTError (status DD_ERR_BUSY / DD_ERR_TOO_LARGE / ...) on refusal.

    The server keeps x and X alive until the ticket's result is taken
    (dense_dft_wait, or dense_dft_poll once done).  Its streams are not ordered
    after torch's: x must already hold its samples (synchronise the stream
    that wrote it before submitting), and X is complete when the result says
    done."""
    d = _one_desc(desc)
    t = _u64()
    if t_arrival_ns is None:
        rc = _lib.dense_dft_submit(server.handle, ctypes.byref(d), ctypes.byref(t))
    else:
        rc = _lib.dense_dft_submit_at(server.handle, ctypes.byref(d), int(t_arrival_ns), ctypes.byref(t))
    _check(rc, "dense_dft_submit")
    if not isinstance(desc, dd_desc):
        server.pending[int(t.value)] = _desc_tensors([desc])
    return int(t.value)


def dense_dft_submit_at(server: Server, desc, t_arrival_ns: int) -> int:
    """Queue one request stamped with the caller's arrival time (open-loop load)."""
    return dense_dft_submit(server, desc, t_arrival_ns)


def dense_dft_submit_many_at(server: Server, descs, t_arrival_ns):
    """Open-loop replay: queue descs[i] at host time t_arrival_ns[i] (non-decreasing,
    dense_dft_clock_ns scale); returns the tickets.  Blocks until the last is queued."""
    descs = list(descs)
    arr, n = _desc_array(descs)
    ts = (_u64 * n)(*[int(t) for t in t_arrival_ns])
    tk = (_u64 * n)()
    done = ctypes.c_int32()
    rc = _lib.dense_dft_submit_many_at(server.handle, arr, ts, n, tk, ctypes.byref(done))
    for i in range(done.value):
        if not isinstance(descs[i], dd_desc):
            server.pending[int(tk[i])] = _desc_tensors([descs[i]])
    _check(rc, f"dense_dft_submit_many_at (queued {done.value} of {n})")
    return [int(t) for t in tk]


def _result_dict(r: dd_result) -> dict:
    return {"status": int(r.status), "batch_requests": int(r.batch_requests), "t_arrival_ns": int(r.t_arrival_ns),
            "t_start_ns": int(r.t_start_ns), "t_done_ns": int(r.t_done_ns)}


def dense_dft_poll(server: Server, ticket: int):
    """Result dict once done (the ticket is then retired), None while pending."""
    r = dd_result()
    rc = _lib.dense_dft_poll(server.handle, int(ticket), ctypes.byref(r))
    if rc == DD_ERR_BUSY:
        return None
    _check(rc, "dense_dft_poll")
    server.pending.pop(int(ticket), None)
    return _result_dict(r)


def dense_dft_wait(server: Server, ticket: int, timeout_us: int = -1) -> dict:
    r = dd_result()
    _check(_lib.dense_dft_wait(server.handle, int(ticket), int(timeout_us), ctypes.byref(r)), "dense_dft_wait")
    server.pending.pop(int(ticket), None)
    return _result_dict(r)


def dense_dft_server_pause(server: Server, paused: bool) -> None:
    _check(_lib.dense_dft_server_pause(server.handle, 1 if paused else 0), "dense_dft_server_pause")


def dense_dft_server_stats(server: Server) -> dict:
    st = dd_server_stats()
    _check(_lib.dense_dft_server_stats(server.handle, ctypes.byref(st)), "dense_dft_server_stats")
    return {name: int(getattr(st, name)) for name, _ in dd_server_stats._fields_}


def dense_dft_server_destroy(server: Server) -> None:
    if server.handle:
        _check(_lib.dense_dft_server_destroy(server.handle), "dense_dft_server_destroy")
        server.handle = None
        server.pending.clear()


def dense_dft_clock_ns() -> int:
    return int(_lib.dense_dft_clock_ns())


# --- torch conveniences (memory allocation only) ---
def dtype_code(torch_dtype) -> int:
    import torch
    m = {torch.float32: DD_F32, torch.complex64: DD_C64, torch.float64: DD_F64,
         torch.complex128: DD_C128}
    if torch_dtype not in m:
        raise TypeError(f"unsupported input dtype {torch_dtype}")
    return m[torch_dtype]


def out_dtype(code: int):
    import torch
    return torch.complex64 if code in (DD_F32, DD_C64) else torch.complex128


def dense_dft_plan_decimated(N: int, p: int, T: float, batch: int, dtype: int,
                             flags: int = DD_TWIDDLE_FP64) -> Plan:
    """Plan of the alpha = 1/p transform (N samples to N/p bins)."""
    h = _vp()
    _check(_lib.dense_dft_plan_decimated(ctypes.byref(h), int(N), int(p), float(T), int(batch), int(dtype),
                                         int(flags)), "dense_dft_plan_decimated")
    plan = Plan(h, N, 1, T, batch, dtype, flags)
    plan.p = int(p)
    return plan


def decimated_dft(x, p: int, T: float, flags: int = DD_TWIDDLE_FP64, plan: Plan | None = None):
    """X = the alpha = 1/p transform of the rows of device tensor x ([batch, N] or [N])."""
    import torch
    squeeze = x.dim() == 1
    x2 = (x.reshape(1, -1) if squeeze else x).contiguous()
    batch, N = x2.shape
    code = dtype_code(x2.dtype)
    if plan is None:
        plan = dense_dft_plan_decimated(N, p, T, batch, code, flags)
    X = torch.empty((batch, N // p), dtype=out_dtype(code), device=x2.device)
    dense_dft_exec(plan, x2, X)
    return X[0] if squeeze else X


def dense_dft_exec_inverse(plan: Plan, X, x, workspace=None, stream=None) -> None:
    """Inverse transform of device spectra X ([batch][alpha*N]) into x ([batch][N] complex)."""
    if not getattr(plan, "p", 0):  # (alpha = 1/p plans are refused by the library: one-way)
        _check_buf(X, "X", out_dtype(plan.dtype), plan.batch * plan.alpha * plan.N)
        _check_buf(x, "x", out_dtype(plan.dtype), plan.batch * plan.N)
        _check_workspace(plan, workspace)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(X.device).cuda_stream
    ws = None if workspace is None else workspace.data_ptr()
    _check(_lib.dense_dft_exec_inverse(plan.handle, X.data_ptr(), x.data_ptr(), ws, _vp(stream)),
           "dense_dft_exec_inverse")


def alpha_idft(X, alpha: int, T: float, flags: int = DD_TWIDDLE_FP64, plan: Plan | None = None):
    """x = inverse alpha-dense DFT of the rows of device tensor X ([batch, alpha*N] or [alpha*N],
    complex64 or complex128): x_n = (1/(alpha T)) sum_m X_m exp(+2 pi i m n/(alpha N)), n < N."""
    import torch
    squeeze = X.dim() == 1
    X2 = (X.reshape(1, -1) if squeeze else X).contiguous()
    batch, M = X2.shape
    if M % alpha:
        raise ValueError("the spectrum length must be a multiple of alpha")
    N = M // alpha
    code = DD_C64 if X2.dtype == torch.complex64 else DD_C128 if X2.dtype == torch.complex128 else None
    if code is None:
        raise TypeError(f"unsupported spectrum dtype {X2.dtype}")
    if plan is None:
        plan = dense_dft_plan(N, alpha, T, batch, code, flags)
    x = torch.empty((batch, N), dtype=X2.dtype, device=X2.device)
    dense_dft_exec_inverse(plan, X2, x)
    return x[0] if squeeze else x


def alpha_dft(x, alpha: int, T: float, flags: int = DD_TWIDDLE_FP64, plan: Plan | None = None):
    """X = alpha-dense DFT of the rows of device tensor x ([batch, N] or [N])."""
    import torch
    squeeze = x.dim() == 1
    x2 = x.reshape(1, -1) if squeeze else x
    x2 = x2.contiguous()
    batch, N = x2.shape
    code = dtype_code(x2.dtype)
    if plan is None:
        plan = dense_dft_plan(N, alpha, T, batch, code, flags)
    X = torch.empty((batch, alpha * N), dtype=out_dtype(code), device=x2.device)
    dense_dft_exec(plan, x2, X)
    return X[0] if squeeze else X
