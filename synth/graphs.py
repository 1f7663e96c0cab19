"""Seeded generators for the synthetic signed bipartite workloads.

Every generator is a pure function of its seed, returns edges as ``int32``
vertex ids (U and V in separate id spaces) and ``int8`` signs in {+1, -1},
and never emits a duplicate (u, v) pair.  The sampling runs in ``gen.c``
(counter-based SplitMix64, Walker alias tables, a hash set for repeats);
per-graph parameters of the batched and served workloads are drawn with
NumPy ``SeedSequence``/``PCG64``.

The workloads stand in for the paper's real datasets (Section V, Table I:
27 K to 257 M edges, heavy-tailed degrees, 30 % negative edges where signs
were assigned at random).  The recipes:

* uniform: ``m`` distinct pairs drawn uniformly from U x V (repeats
  rejected); each sign is -1 with probability ``q``.
* Chung-Lu bipartite: per side, weights ``w = (1 - xi) ** (-1 / (gamma - 1))``
  with ``xi ~ U[0, 1)`` (a Pareto law whose degree density falls as
  ``d ** -gamma``), clipped so that the expected degree ``m * w / sum(w)``
  is at most ``d_cap``, then renormalised once.  Pairs (u ~ w_U, v ~ w_V) are
  drawn one after another; repeats are dropped and the first ``m`` distinct
  pairs in draw order are kept.  Signs are then drawn i.i.d., -1 with
  probability ``q``.
"""

from __future__ import annotations

from dataclasses import dataclass
import ctypes
import math
import os
import subprocess

import numpy as np


@dataclass
class SignedGraph:
    """An edge list of a signed bipartite graph."""

    n_u: int
    n_v: int
    u: np.ndarray  # int32 [m], ids in [0, n_u)
    v: np.ndarray  # int32 [m], ids in [0, n_v)
    sign: np.ndarray  # int8 [m], +1 or -1
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.u.shape[0])


_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``gen.c`` into ``libsynth.so`` (plain C, gcc)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = f"{_LIB}.tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, f64, u64, p = ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p
        lib.synth_chung_lu.restype = i64
        lib.synth_chung_lu.argtypes = [i64, i64, i64, f64, f64, f64, f64, f64, u64, i64, p, p, p]
        lib.synth_uniform.restype = i64
        lib.synth_uniform.argtypes = [i64, i64, i64, f64, u64, p, p, p]
        _lib = lib
    return _lib


def _alloc(m: int):
    return (np.empty(m, np.int32), np.empty(m, np.int32), np.empty(m, np.int8))


def _seed64(seed) -> int:
    return int(seed) & 0xFFFFFFFFFFFFFFFF


def uniform_graph(n_u: int, n_v: int, m: int, q: float, seed=0, name="") -> SignedGraph:
    """``m`` distinct pairs uniform over U x V, signs -1 with probability ``q``."""
    m = int(min(m, n_u * n_v))
    u, v, s = _alloc(m)
    rc = _load().synth_uniform(n_u, n_v, m, q, _seed64(seed),
                               u.ctypes.data, v.ctypes.data, s.ctypes.data)
    if rc != m:
        raise RuntimeError(f"synth_uniform failed ({rc})")
    return SignedGraph(n_u, n_v, u, v, s, name)


def chung_lu_graph(n_u: int, n_v: int, m: int, gamma_u: float, gamma_v: float,
                   q: float, d_cap_u=None, d_cap_v=None, seed=0, name="",
                   max_draw_factor: int = 4096) -> SignedGraph:
    """Chung-Lu bipartite graph with Pareto expected degrees (see module doc).

    ``d_cap_u`` / ``d_cap_v`` bound the expected degree on U / V; by default
    they are the size of the other side.  ``m`` is clipped to ``n_u * n_v``.
    """
    m = int(min(m, n_u * n_v))
    d_cap_u = float(n_v if d_cap_u is None else d_cap_u)
    d_cap_v = float(n_u if d_cap_v is None else d_cap_v)
    u, v, s = _alloc(m)
    rc = _load().synth_chung_lu(n_u, n_v, m, gamma_u, gamma_v, q, d_cap_u, d_cap_v,
                                _seed64(seed), max_draw_factor * max(m, 1024),
                                u.ctypes.data, v.ctypes.data, s.ctypes.data)
    if rc != m:
        raise RuntimeError(f"synth_chung_lu({n_u}, {n_v}, {m}) failed ({rc})")
    return SignedGraph(n_u, n_v, u, v, s, name)


# --- the named workloads -----------------------------------------------------

CONFIGS = {
    "tiny": dict(kind="uniform", n_u=2_000, n_v=1_500, m=20_000, q=0.3, seed=0),
    "powerlaw2m": dict(kind="chung_lu", n_u=200_000, n_v=100_000, m=2_000_000,
                       gamma_u=2.3, gamma_v=2.1, q=0.25, seed=0),
    "skewed50m": dict(kind="chung_lu", n_u=5_000_000, n_v=2_000_000, m=50_000_000,
                      gamma_u=2.1, gamma_v=1.9, q=0.4, d_cap_u=100_000,
                      d_cap_v=100_000, seed=0),
    # stand-ins for the two datasets of the wedge-separation study (Section V,
    # Table IV; Table I: SE 27,083 edges, 15.32 M balanced butterflies; HO
    # 114,378 edges, 280.79 M): same edge counts, heavy-tailed degrees tuned
    # to a similar number of balanced butterflies (14.0 M and 345 M), 30 %
    # negative edges
    "se_like": dict(kind="chung_lu", n_u=6_000, n_v=2_000, m=27_083,
                    gamma_u=2.1, gamma_v=1.7, q=0.3, seed=0),
    "ho_like": dict(kind="chung_lu", n_u=20_000, n_v=5_000, m=114_378,
                    gamma_u=2.0, gamma_v=1.6, q=0.3, seed=0),
}


def config_graph(name: str, scale: float = 1.0, seed=None, q=None) -> SignedGraph:
    """One of the named single-graph workloads; ``scale`` shrinks it for tests
    (sizes and edge count multiplied by ``scale``, degree caps unchanged);
    ``q`` replaces the negative-sign probability.  Signs are drawn from a
    stream of their own after the topology, so the same seed with another
    ``q`` gives the same edges with other signs."""
    c = dict(CONFIGS[name])
    kind = c.pop("kind")
    if seed is not None:
        c["seed"] = seed
    if q is not None:
        c["q"] = float(q)
    if scale != 1.0:
        for k in ("n_u", "n_v", "m"):
            c[k] = max(4, int(round(c[k] * scale)))
        if "d_cap_u" in c:
            c["d_cap_u"] = min(c["d_cap_u"], c["n_v"])
            c["d_cap_v"] = min(c["d_cap_v"], c["n_u"])
    if kind == "uniform":
        return uniform_graph(name=name, **c)
    return chung_lu_graph(name=name, **c)


def batch_graph(i: int, n_graphs: int = 4096, seed: int = 0) -> SignedGraph:
    """Graph ``i`` of the batched workload: 4,096 graphs from
    ``SeedSequence(seed).spawn(4096)``; |U|, |V| uniform in [50, 5000], m
    uniform in [200, 50000] clipped to floor(|U||V| / 2), Chung-Lu exponent
    2.2 on both sides, negative probability uniform in [0.1, 0.5]."""
    return _batch_like(np.random.SeedSequence(seed).spawn(n_graphs)[i], f"batch{i}")


def _batch_like(ss, name: str) -> SignedGraph:
    rng = np.random.Generator(np.random.PCG64(ss))
    n_u = int(rng.integers(50, 5001))
    n_v = int(rng.integers(50, 5001))
    m = int(rng.integers(200, 50001))
    m = min(m, (n_u * n_v) // 2)
    q = float(rng.uniform(0.1, 0.5))
    sub = int(rng.integers(0, 2**63 - 1))
    return chung_lu_graph(n_u, n_v, m, 2.2, 2.2, q, seed=sub, name=name)


def batch_graphs(n_graphs: int = 4096, seed: int = 0, first: int = 0, count=None):
    """Graphs first .. first + count - 1 of the batched workload (the same
    graphs as batch_graph, with the seed sequence spawned once)."""
    count = n_graphs - first if count is None else count
    kids = np.random.SeedSequence(seed).spawn(n_graphs)
    return [_batch_like(kids[i], f"batch{i}") for i in range(first, first + count)]


def pool_graph(i: int, n_pool: int = 1000, seed: int = 0) -> SignedGraph:
    """Graph ``i`` of the serving pool: m log-uniform on [1e3, 5e6],
    |U| = m // 10, |V| = m // 20, exponent 2.2, negative probability 0.3."""
    ss = np.random.SeedSequence(seed).spawn(n_pool)[i]
    return _pool_like(ss, f"pool{i}")


def pool_graphs(n_pool: int = 1000, seed: int = 0, idx=None):
    """Graphs idx (default: all) of the serving pool, the seed sequence
    spawned once; the same graphs as pool_graph."""
    kids = np.random.SeedSequence(seed).spawn(n_pool)
    idx = range(n_pool) if idx is None else idx
    return [_pool_like(kids[i], f"pool{i}") for i in idx]


def upload_graph(j: int, seed: int = 1) -> SignedGraph:
    """Graph ``j`` of the newly uploaded stream (same law as the pool)."""
    ss = np.random.SeedSequence([seed, j])
    return _pool_like(ss, f"upload{j}")


def _pool_like(ss, name: str, m_lo: float = 1e3, m_hi: float = 5e6) -> SignedGraph:
    rng = np.random.Generator(np.random.PCG64(ss))
    m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
    n_u = max(2, m // 10)
    n_v = max(2, m // 20)
    m = min(m, (n_u * n_v) // 2)
    sub = int(rng.integers(0, 2**63 - 1))
    return chung_lu_graph(n_u, n_v, m, 2.2, 2.2, 0.3, seed=sub, name=name)
