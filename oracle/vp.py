"""Python front of the vertex-priority oracle in ``vp.c`` (test infrastructure only).

``vp.c`` is built with gcc into ``libdbbc_oracle.so`` beside it; nothing in
the GPU library links or loads it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vp.c")
_LIB = os.path.join(_HERE, "libdbbc_oracle.so")
_lib = None


class _Counts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("balanced", "unbalanced", "total", "wedges", "expansions")]


@dataclass
class OracleResult:
    balanced: int
    unbalanced: int
    total: int
    wedges: int
    expansions: int
    per_pivot_bal: np.ndarray | None = None
    bal_u: np.ndarray | None = None
    bal_v: np.ndarray | None = None
    unb_u: np.ndarray | None = None
    unb_v: np.ndarray | None = None
    bal_e: np.ndarray | None = None
    unb_e: np.ndarray | None = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11 + pthreads)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = f"{_LIB}.tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", "-pthread",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _declare(lib):
    i64, p = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_vp_count.restype = ctypes.c_int
    lib.oracle_vp_count.argtypes = [i64, i64, i64, p, p, p, p, ctypes.c_int, p, i64,
                                    p, p, p, p, p, ctypes.POINTER(_Counts)]
    if hasattr(lib, "oracle_graph_build"):
        lib.oracle_graph_build.restype = p
        lib.oracle_graph_build.argtypes = [i64, i64, i64, p, p, p, p]
        lib.oracle_graph_count.restype = ctypes.c_int
        lib.oracle_graph_count.argtypes = [p, ctypes.c_int, p, i64, p, p, p, p, p,
                                           ctypes.POINTER(_Counts)]
        lib.oracle_graph_free.restype = None
        lib.oracle_graph_free.argtypes = [p]
    return lib


def _load(lib_path=None):
    """The oracle library; ``lib_path`` loads another build of the same
    source (the mutation tests compile deliberately broken copies)."""
    global _lib
    if lib_path is not None:
        return _declare(ctypes.CDLL(lib_path))
    if _lib is None:
        _lib = _declare(ctypes.CDLL(build()))
    return _lib


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def vp_counts(n_u, n_v, u, v, sign, ids=None, threads=None, pivots=None,
              per_pivot=False, per_vertex=False, per_edge=False, lib_path=None) -> OracleResult:
    """Algorithm 1 Phase 5 over the whole graph (or over ``pivots``, global
    indices: U vertex x is x, V vertex y is n_u + y).  ``ids`` overrides the
    tie-break id of Definition 3 per global index.  ``per_edge`` adds, per
    input record, the balanced and unbalanced butterflies containing it
    (``bal_e``, ``unb_e``); records must name distinct (u, v) pairs."""
    lib = _load(lib_path)
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    s = np.ascontiguousarray(sign, dtype=np.int8)
    m = int(u.shape[0])
    n = int(n_u) + int(n_v)
    keep = []

    def ptr(a):
        if a is None:
            return None
        keep.append(a)
        return a.ctypes.data

    id_arr = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
    piv = None if pivots is None else np.ascontiguousarray(pivots, dtype=np.int32)
    ppb = np.zeros(n, np.int64) if per_pivot else None
    bal = np.zeros(n, np.int64) if per_vertex else None
    unb = np.zeros(n, np.int64) if per_vertex else None
    bal_e = np.zeros(m, np.int64) if per_edge else None
    unb_e = np.zeros(m, np.int64) if per_edge else None
    out = _Counts()
    rc = lib.oracle_vp_count(int(n_u), int(n_v), m, ptr(u), ptr(v), ptr(s), ptr(id_arr),
                             int(threads or default_threads()), ptr(piv),
                             0 if piv is None else int(piv.shape[0]),
                             ptr(ppb), ptr(bal), ptr(unb), ptr(bal_e), ptr(unb_e),
                             ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_vp_count rejected the graph")
    res = OracleResult(out.balanced, out.unbalanced, out.total, out.wedges, out.expansions)
    if per_pivot:
        res.per_pivot_bal = ppb
    if per_vertex:
        res.bal_u, res.bal_v = bal[:n_u], bal[n_u:]
        res.unb_u, res.unb_v = unb[:n_u], unb[n_u:]
    if per_edge:
        res.bal_e, res.unb_e = bal_e, unb_e
    return res


class OracleGraph:
    """The oracle's adjacency lists, built once (``oracle_graph_build``), so
    that Phase 5 alone (``count``) can be run and timed apart from the
    build."""

    def __init__(self, n_u, n_v, u, v, sign):
        self._lib = _load()
        self.n_u, self.n_v = int(n_u), int(n_v)
        u = np.ascontiguousarray(u, dtype=np.int32)
        v = np.ascontiguousarray(v, dtype=np.int32)
        s = np.ascontiguousarray(sign, dtype=np.int8)
        self.m = int(u.shape[0])
        self._h = self._lib.oracle_graph_build(self.n_u, self.n_v, self.m, u.ctypes.data,
                                               v.ctypes.data, s.ctypes.data, None)
        if not self._h:
            raise ValueError("oracle_graph_build rejected the graph")

    def count(self, threads=None, pivots=None) -> OracleResult:
        """Phase 5 over every pivot, or over ``pivots`` (global indices)."""
        piv = None if pivots is None else np.ascontiguousarray(pivots, dtype=np.int32)
        out = _Counts()
        rc = self._lib.oracle_graph_count(self._h, int(threads or default_threads()),
                                          None if piv is None else piv.ctypes.data,
                                          0 if piv is None else int(piv.shape[0]),
                                          None, None, None, None, None, ctypes.byref(out))
        if rc != 0:
            raise ValueError("oracle_graph_count rejected its arguments")
        return OracleResult(out.balanced, out.unbalanced, out.total, out.wedges, out.expansions)

    def close(self):
        if self._h:
            self._lib.oracle_graph_free(self._h)
            self._h = None

    def __del__(self):
        self.close()
