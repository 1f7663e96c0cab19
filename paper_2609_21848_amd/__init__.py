"""Python binding of libdbbc: exact balanced / unbalanced butterfly counts in
signed bipartite graphs on AMD MI355X (gfx950).

Every function below marshals arguments for the C entry point of the same
name in ``include/dbbc.h`` and raises ``DbbcError`` on a non-zero status.
All counting runs in the HIP kernels of ``libdbbc.so``; this module never
computes counts itself.  PyTorch is used only for device tensors and streams.
"""

from __future__ import annotations

import ctypes
import os
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdbbc.so")

DBBC_OK = 0
DBBC_E_INVALID_ARG = -1
DBBC_E_ID_RANGE = -2
DBBC_E_SIGN = -3
DBBC_E_DUPLICATE = -4
DBBC_E_OOM = -5
DBBC_E_DEVICE = -6
DBBC_E_TOO_LARGE = -7
DBBC_E_NO_DEVICE = -8
DBBC_E_PARSE = -9

DBBC_INPUT_DEVICE = 0x1
DBBC_DUP_REJECT = 0x2
DBBC_OPT_TIME_KERNELS = 0x1
DBBC_OPT_WIDE_EDGES = 0x2
DBBC_OPT_HOST_PLAN = 0x4
DBBC_BATCH_CAPTURE = 0x1
DBBC_SERVER_NO_MERGE = 0x1

# every symbol declared in include/dbbc.h
EXPORTS = (
    "dbbc_graph_create", "dbbc_graph_stats", "dbbc_count", "dbbc_count_async", "dbbc_count_read",
    "dbbc_count_per_vertex", "dbbc_count_per_edge", "dbbc_graph_create_text", "dbbc_graph_raw_ids",
    "dbbc_count_explicit",
    "dbbc_batch_create", "dbbc_batch_reset", "dbbc_batch_launch",
    "dbbc_batch_read",
    "dbbc_batch_count", "dbbc_batch_size", "dbbc_batch_destroy", "dbbc_count_batch", "dbbc_autotune",
    "dbbc_last_kernel_times", "dbbc_graph_destroy", "dbbc_status_string", "dbbc_last_error",
    "dbbc_version", "dbbc_graph_plan", "dbbc_now_ns", "dbbc_server_create", "dbbc_server_add_graph",
    "dbbc_server_submit", "dbbc_server_submit_upload", "dbbc_server_wait", "dbbc_server_get_stats",
    "dbbc_server_last_error", "dbbc_server_destroy", "dbbc_count_noalloc",
)


class DbbcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Counts(NamedTuple):
    balanced: int
    unbalanced: int
    total: int
    wedges: int


class _Counts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("balanced", "unbalanced", "total", "wedges")]


class _Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "n_u", "n_v", "m", "dups_dropped", "max_deg_u", "max_deg_v", "device_bytes",
        "wedges_vp", "pivots_active")]


class Options(ctypes.Structure):
    """Mirror of dbbc_options; -1 leaves a knob at the library default."""
    _fields_ = [("hub_T", ctypes.c_int32), ("window_L", ctypes.c_int32),
                ("reverse_L", ctypes.c_int32), ("small_work", ctypes.c_int32),
                ("part_work", ctypes.c_int32), ("long_len", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]

    def __init__(self, hub_T=-1, window_L=-1, small_work=-1, part_work=-1, flags=0,
                 reverse_L=-1, long_len=-1):
        super().__init__(hub_T, window_L, reverse_L, small_work, part_work, long_len, flags)


class ServerConfig(ctypes.Structure):
    """Mirror of dbbc_server_config (zero = default)."""
    _fields_ = [("hbm_budget", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("solo_wedges", ctypes.c_int64),
                ("batch_wedges", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("graph_id", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("queued_ahead", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_int64), ("t_launch_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "completed", "failed", "rejected", "uploads", "evicted", "launches",
        "batched_graphs", "max_queue", "queued", "resident_graphs", "resident_bytes")]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """Mirror of dbbc_allocator: the device allocator of a graph handle."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


_torch_alloc = None


def torch_allocator() -> Allocator:
    """A dbbc_allocator that takes the library's device memory from PyTorch's
    caching allocator (``torch.cuda.caching_allocator_alloc`` on the stream
    the library names) and gives it back with ``caching_allocator_delete``.
    One shared instance; its callbacks stay alive with the module."""
    global _torch_alloc
    if _torch_alloc is None:
        import torch

        def _alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                          int(stream or 0))
            except Exception:  # out of memory: the library reports DBBC_E_OOM
                return None

        def _free(ptr, stream, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        _torch_alloc = Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)
    return _torch_alloc


def _allocator_arg(allocator):
    """ctypes argument for an allocator choice: "torch" (PyTorch's caching
    allocator), None / "hip" (hipMalloc), or an Allocator."""
    if allocator == "torch":
        return ctypes.byref(torch_allocator())
    if allocator is None or allocator == "hip":
        return None
    if isinstance(allocator, Allocator):
        return ctypes.byref(allocator)
    raise ValueError(f"unknown allocator {allocator!r}")


class _TextInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("lines", "records", "n_u", "n_v")]


class _KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("ms", ctypes.c_float), ("wedges", ctypes.c_int64),
                ("segments", ctypes.c_int64), ("items", ctypes.c_int64), ("macs", ctypes.c_int64)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdbbc.so (built by ``paper_2609_21848_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2609_21848_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.dbbc_graph_create.argtypes = [i32, i32, i64, vp, vp, vp, u32, vp, vp, ctypes.POINTER(vp)]
    lib.dbbc_graph_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
    lib.dbbc_count.argtypes = [vp, ctypes.POINTER(Options), ctypes.POINTER(_Counts), vp]
    lib.dbbc_count_per_vertex.argtypes = [vp, ctypes.POINTER(Options), vp, vp, vp, vp,
                                          ctypes.POINTER(_Counts), vp]
    lib.dbbc_count_per_edge.argtypes = [vp, ctypes.POINTER(Options), vp, vp,
                                        ctypes.POINTER(_Counts), vp]
    lib.dbbc_graph_create_text.argtypes = [vp, i64, u32, vp, vp, ctypes.POINTER(vp),
                                           ctypes.POINTER(_TextInfo)]
    lib.dbbc_graph_raw_ids.argtypes = [vp, i32, vp, vp]
    lib.dbbc_count_explicit.argtypes = [vp, ctypes.POINTER(_Counts), vp]
    lib.dbbc_count_async.argtypes = [vp, ctypes.POINTER(Options), vp]
    lib.dbbc_count_noalloc.argtypes = [vp, ctypes.POINTER(Options), ctypes.POINTER(_Counts), vp]
    lib.dbbc_count_read.argtypes = [vp, ctypes.POINTER(_Counts)]
    lib.dbbc_batch_create.argtypes = [vp, i32, ctypes.POINTER(Options), u32, vp, ctypes.POINTER(vp)]
    lib.dbbc_batch_reset.argtypes = [vp, vp, i32, ctypes.POINTER(Options), u32, vp]
    lib.dbbc_batch_launch.argtypes = [vp, vp]
    lib.dbbc_batch_read.argtypes = [vp, ctypes.POINTER(_Counts)]
    lib.dbbc_batch_count.argtypes = [vp, ctypes.POINTER(_Counts), vp]
    lib.dbbc_batch_size.argtypes = [vp]
    lib.dbbc_batch_size.restype = i32
    lib.dbbc_batch_destroy.argtypes = [vp]
    lib.dbbc_batch_destroy.restype = None
    lib.dbbc_count_batch.argtypes = [vp, i32, ctypes.POINTER(Options), ctypes.POINTER(_Counts), vp]
    lib.dbbc_autotune.argtypes = [vp, i32, ctypes.POINTER(Options), i32, vp, ctypes.POINTER(Options),
                                  ctypes.POINTER(ctypes.c_float)]
    lib.dbbc_last_kernel_times.argtypes = [vp, ctypes.POINTER(_KernelTime), i32,
                                           ctypes.POINTER(i32)]
    lib.dbbc_graph_plan.argtypes = [vp, ctypes.POINTER(Options), vp]
    lib.dbbc_now_ns.restype = i64
    lib.dbbc_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(Options),
                                       ctypes.POINTER(vp)]
    lib.dbbc_server_add_graph.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.POINTER(i32)]
    lib.dbbc_server_submit.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.dbbc_server_submit_upload.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.POINTER(i64)]
    lib.dbbc_server_wait.argtypes = [vp, i64, ctypes.POINTER(_Counts), ctypes.POINTER(RequestInfo)]
    lib.dbbc_server_get_stats.argtypes = [vp, ctypes.POINTER(_ServerStats)]
    lib.dbbc_server_last_error.restype = ctypes.c_char_p
    lib.dbbc_server_destroy.argtypes = [vp]
    lib.dbbc_server_destroy.restype = None
    lib.dbbc_graph_destroy.argtypes = [vp]
    lib.dbbc_graph_destroy.restype = None
    lib.dbbc_status_string.argtypes = [ctypes.c_int]
    lib.dbbc_status_string.restype = ctypes.c_char_p
    lib.dbbc_last_error.restype = ctypes.c_char_p
    lib.dbbc_version.restype = ctypes.c_char_p
    for name in ("dbbc_graph_create", "dbbc_graph_stats", "dbbc_count", "dbbc_count_async",
                 "dbbc_count_read", "dbbc_count_per_vertex", "dbbc_count_per_edge",
                 "dbbc_graph_create_text", "dbbc_graph_raw_ids", "dbbc_count_explicit",
                 "dbbc_batch_create", "dbbc_batch_reset",
                 "dbbc_batch_launch",
                 "dbbc_batch_read", "dbbc_batch_count", "dbbc_count_batch", "dbbc_autotune",
                 "dbbc_last_kernel_times", "dbbc_graph_plan", "dbbc_server_create",
                 "dbbc_server_add_graph", "dbbc_server_submit", "dbbc_server_submit_upload",
                 "dbbc_server_wait", "dbbc_server_get_stats", "dbbc_count_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != DBBC_OK:
        lib = load()
        detail = lib.dbbc_last_error().decode()
        if where.startswith("dbbc_server"):
            detail = lib.dbbc_server_last_error().decode() or detail
        detail = detail or lib.dbbc_status_string(status).decode()
        raise DbbcError(status, where, detail)


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:  # pragma: no cover
            pass
        return None
    return getattr(stream, "cuda_stream", stream)


def _edge_args(u, v, sign):
    """(pointers, flags, keepalive) for host NumPy arrays or torch tensors."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(u, torch.Tensor):
        dev = u.is_cuda
        u = u.to(torch.int32).contiguous()
        v = v.to(device=u.device, dtype=torch.int32).contiguous()
        sign = sign.to(device=u.device, dtype=torch.int8).contiguous()
        flags = DBBC_INPUT_DEVICE if dev else 0
        return (u.data_ptr(), v.data_ptr(), sign.data_ptr()), flags, (u, v, sign), int(u.numel())
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    sign = np.ascontiguousarray(sign, dtype=np.int8)
    return (u.ctypes.data, v.ctypes.data, sign.ctypes.data), 0, (u, v, sign), int(u.shape[0])


def dbbc_graph_create(n_u: int, n_v: int, u, v, sign, flags: int = 0, stream=None,
                      allocator="torch") -> int:
    """Build a handle; u, v, sign as NumPy arrays or torch tensors (device
    tensors set DBBC_INPUT_DEVICE).  ``allocator``: "torch" (the handle's
    device memory from PyTorch's caching allocator), None / "hip"
    (hipMalloc) or an Allocator.  Returns the opaque handle."""
    lib = load()
    ptrs, f, keep, m = _edge_args(u, v, sign)
    if len(np.shape(u)) != 1 or len(keep[1]) != m or len(keep[2]) != m:
        raise ValueError("u, v and sign must be 1-D and of equal length")
    out = ctypes.c_void_p()
    _check(lib.dbbc_graph_create(int(n_u), int(n_v), m, *ptrs, int(flags) | f,
                                 _allocator_arg(allocator), _stream_ptr(stream), ctypes.byref(out)),
           "dbbc_graph_create")
    return out.value


def dbbc_graph_create_text(text, flags: int = 0, stream=None, allocator="torch"):
    """Build a handle from an edge-list text parsed on the device.  text:
    bytes / str (host), or a uint8 CUDA tensor (sets DBBC_INPUT_DEVICE);
    ``allocator`` as for dbbc_graph_create.  Returns (handle, info dict with
    lines, records, n_u, n_v)."""
    lib = load()
    keep = None
    if hasattr(text, "is_cuda") and text.is_cuda:
        if not text.is_contiguous():
            raise ValueError("text tensor must be contiguous")
        ptr, n, flags = text.data_ptr(), int(text.numel() * text.element_size()), flags | DBBC_INPUT_DEVICE
    else:
        keep = np.frombuffer(text.encode() if isinstance(text, str) else bytes(text), dtype=np.uint8)
        ptr, n = (keep.ctypes.data if keep.size else None), int(keep.size)
    out = ctypes.c_void_p()
    info = _TextInfo()
    _check(lib.dbbc_graph_create_text(ptr, n, int(flags), _allocator_arg(allocator), _stream_ptr(stream),
                                      ctypes.byref(out), ctypes.byref(info)), "dbbc_graph_create_text")
    return out.value, {k: int(getattr(info, k)) for k, _ in _TextInfo._fields_}


def dbbc_graph_stats(g: int) -> dict:
    s = _Stats()
    _check(load().dbbc_graph_stats(g, ctypes.byref(s)), "dbbc_graph_stats")
    return {k: int(getattr(s, k)) for k, _ in _Stats._fields_}


def dbbc_count(g: int, options: Options | None = None, stream=None) -> Counts:
    c = _Counts()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_count(g, opt, ctypes.byref(c), _stream_ptr(stream)), "dbbc_count")
    return Counts(c.balanced, c.unbalanced, c.total, c.wedges)


def dbbc_count_noalloc(g: int, options: Options | None = None, stream=None) -> Counts:
    """dbbc_count on a graph already planned for ``options``, with no
    allocation (its scratch is the library's per-GPU static array)."""
    c = _Counts()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_count_noalloc(g, opt, ctypes.byref(c), _stream_ptr(stream)), "dbbc_count_noalloc")
    return Counts(c.balanced, c.unbalanced, c.total, c.wedges)


def dbbc_count_async(g: int, options: Options | None = None, stream=None) -> None:
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_count_async(g, opt, _stream_ptr(stream)), "dbbc_count_async")


def dbbc_count_read(g: int) -> Counts:
    c = _Counts()
    _check(load().dbbc_count_read(g, ctypes.byref(c)), "dbbc_count_read")
    return Counts(c.balanced, c.unbalanced, c.total, c.wedges)


def _out_ptr(t):
    if t is None:
        return None
    if t.dtype != __import__("torch").int64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("per-vertex and per-edge outputs must be contiguous int64 CUDA tensors")
    return t.data_ptr()


def dbbc_count_per_vertex(g: int, bal_u=None, bal_v=None, unb_u=None, unb_v=None,
                          options: Options | None = None, stream=None) -> Counts:
    """Fill caller-owned int64 device tensors (any may be None)."""
    p = _out_ptr
    c = _Counts()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_count_per_vertex(g, opt, p(bal_u), p(bal_v), p(unb_u), p(unb_v),
                                        ctypes.byref(c), _stream_ptr(stream)),
           "dbbc_count_per_vertex")
    return Counts(c.balanced, c.unbalanced, c.total, c.wedges)


def dbbc_count_per_edge(g: int, bal_e=None, unb_e=None, options: Options | None = None,
                        stream=None) -> Counts:
    """Fill caller-owned int64 device tensors of one entry per input record
    (either may be None)."""
    c = _Counts()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_count_per_edge(g, opt, _out_ptr(bal_e), _out_ptr(unb_e), ctypes.byref(c),
                                      _stream_ptr(stream)), "dbbc_count_per_edge")
    return Counts(c.balanced, c.unbalanced, c.total, c.wedges)


def _handles(gs):
    hs = [getattr(g, "handle", g) for g in gs]
    return (ctypes.c_void_p * max(len(hs), 1))(*hs), len(hs)


def dbbc_batch_create(gs, options: Options | None = None, flags: int = 0, stream=None) -> int:
    arr, k = _handles(gs)
    out = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_batch_create(arr, k, opt, int(flags), _stream_ptr(stream), ctypes.byref(out)),
           "dbbc_batch_create")
    return out.value


def dbbc_batch_reset(b: int, gs, options: Options | None = None, flags: int = 0, stream=None) -> None:
    arr, k = _handles(gs)
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_batch_reset(b, arr, k, opt, int(flags), _stream_ptr(stream)), "dbbc_batch_reset")


def dbbc_batch_launch(b: int, stream=None) -> None:
    _check(load().dbbc_batch_launch(b, _stream_ptr(stream)), "dbbc_batch_launch")


def dbbc_batch_read(b: int) -> list:
    k = load().dbbc_batch_size(b)
    out = (_Counts * max(k, 1))()
    _check(load().dbbc_batch_read(b, out), "dbbc_batch_read")
    return [Counts(c.balanced, c.unbalanced, c.total, c.wedges) for c in out[:k]]


def dbbc_batch_count(b: int, stream=None) -> list:
    k = load().dbbc_batch_size(b)
    out = (_Counts * max(k, 1))()
    _check(load().dbbc_batch_count(b, out, _stream_ptr(stream)), "dbbc_batch_count")
    return [Counts(c.balanced, c.unbalanced, c.total, c.wedges) for c in out[:k]]


def dbbc_batch_destroy(b: int) -> None:
    if b:
        load().dbbc_batch_destroy(b)


def dbbc_count_batch(gs, options: Options | None = None, stream=None) -> list:
    arr, k = _handles(gs)
    out = (_Counts * max(k, 1))()
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_count_batch(arr, k, opt, out, _stream_ptr(stream)), "dbbc_count_batch")
    return [Counts(c.balanced, c.unbalanced, c.total, c.wedges) for c in out[:k]]


def dbbc_autotune(gs, start: Options | None = None, reps: int = 3, stream=None):
    """(best options as a dict of the knobs, ms per batch) for graphs gs."""
    arr, k = _handles(gs)
    best = Options()
    ms = ctypes.c_float()
    opt = ctypes.byref(start) if start is not None else None
    _check(load().dbbc_autotune(arr, k, opt, int(reps), _stream_ptr(stream), ctypes.byref(best),
                                ctypes.byref(ms)), "dbbc_autotune")
    knobs = {k: int(getattr(best, k)) for k, _ in Options._fields_ if k != "flags"}
    return knobs, float(ms.value)


def dbbc_last_kernel_times(g: int) -> list:
    """Per-kernel records of the last count run with DBBC_OPT_TIME_KERNELS."""
    buf = (_KernelTime * 16)()
    n = ctypes.c_int32()
    _check(load().dbbc_last_kernel_times(g, buf, 16, ctypes.byref(n)), "dbbc_last_kernel_times")
    return [dict(name=k.name.decode(), ms=float(k.ms), wedges=int(k.wedges),
                 segments=int(k.segments), items=int(k.items), macs=int(k.macs))
            for k in buf[:min(n.value, 16)]]


def dbbc_graph_destroy(g: int) -> None:
    if g:
        load().dbbc_graph_destroy(g)


def dbbc_version() -> str:
    return load().dbbc_version().decode()


class Graph:
    """Owning wrapper: ``with Graph(n_u, n_v, u, v, sign) as g: g.count()``."""

    def __init__(self, n_u, n_v, u, v, sign, flags=0, stream=None, allocator="torch"):
        self.n_u, self.n_v = int(n_u), int(n_v)
        self.m_in = int(len(u))  # input records, duplicates included
        self.handle = None
        self.handle = dbbc_graph_create(n_u, n_v, u, v, sign, flags, stream, allocator)

    def count(self, stream=None, **opts) -> Counts:
        return dbbc_count(self.handle, Options(**opts) if opts else None, stream)

    def count_per_vertex(self, stream=None, **opts):
        """(Counts, bal_u, bal_v, unb_u, unb_v): int64 CUDA tensors in input id order."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        bu = torch.empty(self.n_u, dtype=torch.int64, device=dev)
        bv = torch.empty(self.n_v, dtype=torch.int64, device=dev)
        uu = torch.empty(self.n_u, dtype=torch.int64, device=dev)
        uv = torch.empty(self.n_v, dtype=torch.int64, device=dev)
        c = dbbc_count_per_vertex(self.handle, bu, bv, uu, uv, Options(**opts) if opts else None,
                                  stream)
        return c, bu, bv, uu, uv

    @classmethod
    def from_text(cls, text, flags=0, stream=None, allocator="torch"):
        """A graph read from an edge-list text on the device (ids compacted
        per side; ``raw_ids`` maps them back).  ``info`` holds the line and
        record counts."""
        handle, info = dbbc_graph_create_text(text, flags, stream, allocator)
        g = cls.__new__(cls)
        g.handle = handle
        g.n_u, g.n_v = info["n_u"], info["n_v"]
        g.m_in = info["records"]
        g.info = info
        return g

    def raw_ids(self, side: int, stream=None):
        """int64 CUDA tensor: the raw id of each compact id of a side (0 = U)."""
        import torch
        n = self.n_u if side == 0 else self.n_v
        t = torch.empty(n, dtype=torch.int64, device=torch.device("cuda", torch.cuda.current_device()))
        _check(load().dbbc_graph_raw_ids(self.handle, int(side), t.data_ptr(), _stream_ptr(stream)),
               "dbbc_graph_raw_ids")
        return t

    def count_per_edge(self, stream=None, **opts):
        """(Counts, bal_e, unb_e): int64 CUDA tensors, one entry per input record."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        be = torch.empty(self.m_in, dtype=torch.int64, device=dev)
        ue = torch.empty(self.m_in, dtype=torch.int64, device=dev)
        c = dbbc_count_per_edge(self.handle, be, ue, Options(**opts) if opts else None, stream)
        return c, be, ue

    def count_explicit(self, stream=None) -> Counts:
        """The explicit-verification baseline (every wedge pair checked)."""
        c = _Counts()
        _check(load().dbbc_count_explicit(self.handle, ctypes.byref(c), _stream_ptr(stream)),
               "dbbc_count_explicit")
        return Counts(c.balanced, c.unbalanced, c.total, c.wedges)

    def count_async(self, stream=None, **opts) -> None:
        dbbc_count_async(self.handle, Options(**opts) if opts else None, stream)

    def read(self) -> Counts:
        return dbbc_count_read(self.handle)

    def kernel_times(self) -> list:
        return dbbc_last_kernel_times(self.handle)

    def stats(self) -> dict:
        return dbbc_graph_stats(self.handle)

    def close(self):
        if self.handle:
            dbbc_graph_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owning wrapper of a batch of Graph objects (kept alive by the batch)."""

    def __init__(self, graphs, capture: bool = False, stream=None, **opts):
        self.graphs = list(graphs)
        self.handle = dbbc_batch_create(self.graphs, Options(**opts) if opts else None,
                                        DBBC_BATCH_CAPTURE if capture else 0, stream)

    def count(self, stream=None) -> list:
        return dbbc_batch_count(self.handle, stream)

    def reset(self, graphs, capture: bool = False, stream=None, **opts) -> None:
        self.graphs = list(graphs)
        dbbc_batch_reset(self.handle, self.graphs, Options(**opts) if opts else None,
                         DBBC_BATCH_CAPTURE if capture else 0, stream)

    def launch(self, stream=None) -> None:
        dbbc_batch_launch(self.handle, stream)

    def read(self) -> list:
        return dbbc_batch_read(self.handle)

    def close(self):
        if self.handle:
            dbbc_batch_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dbbc_graph_plan(g: int, options: Options | None = None, stream=None) -> None:
    opt = ctypes.byref(options) if options is not None else None
    _check(load().dbbc_graph_plan(g, opt, _stream_ptr(stream)), "dbbc_graph_plan")


def dbbc_now_ns() -> int:
    return int(load().dbbc_now_ns())


class Server:
    """Owning wrapper of dbbc_server_*: resident graphs and count requests
    answered by the library's scheduler thread (continuous batching)."""

    def __init__(self, hbm_budget=0, slots=0, max_batch=0, solo_wedges=0, batch_wedges=0,
                 merge=True, **opts):
        cfg = ServerConfig(int(hbm_budget), int(slots), int(max_batch), int(solo_wedges),
                           int(batch_wedges), 0 if merge else DBBC_SERVER_NO_MERGE, 0)
        out = ctypes.c_void_p()
        opt = ctypes.byref(Options(**opts)) if opts else None
        _check(load().dbbc_server_create(ctypes.byref(cfg), opt, ctypes.byref(out)),
               "dbbc_server_create")
        self.handle = out.value

    def add_graph(self, n_u, n_v, u, v, sign) -> int:
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        sign = np.ascontiguousarray(sign, dtype=np.int8)
        gid = ctypes.c_int32()
        _check(load().dbbc_server_add_graph(self.handle, int(n_u), int(n_v), len(u), u.ctypes.data,
                                            v.ctypes.data, sign.ctypes.data, ctypes.byref(gid)),
               "dbbc_server_add_graph")
        return gid.value

    def submit(self, graph_id: int) -> int:
        t = ctypes.c_int64()
        _check(load().dbbc_server_submit(self.handle, int(graph_id), ctypes.byref(t)),
               "dbbc_server_submit")
        return t.value

    def submit_upload(self, n_u, n_v, u, v, sign) -> int:
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        sign = np.ascontiguousarray(sign, dtype=np.int8)
        t = ctypes.c_int64()
        _check(load().dbbc_server_submit_upload(self.handle, int(n_u), int(n_v), len(u),
                                                u.ctypes.data, v.ctypes.data, sign.ctypes.data,
                                                ctypes.byref(t)), "dbbc_server_submit_upload")
        return t.value

    def wait(self, ticket: int):
        """(status, Counts or None, info dict) of a request."""
        c = _Counts()
        info = RequestInfo()
        st = load().dbbc_server_wait(self.handle, int(ticket), ctypes.byref(c), ctypes.byref(info))
        d = {k: int(getattr(info, k)) for k, _ in RequestInfo._fields_}
        counts = Counts(c.balanced, c.unbalanced, c.total, c.wedges) if st == DBBC_OK else None
        return st, counts, d

    def stats(self) -> dict:
        s = _ServerStats()
        _check(load().dbbc_server_get_stats(self.handle, ctypes.byref(s)), "dbbc_server_get_stats")
        return {k: int(getattr(s, k)) for k, _ in _ServerStats._fields_}

    def close(self):
        if self.handle:
            load().dbbc_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
