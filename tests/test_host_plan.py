"""CPU checks of the library's host logic: the priority relabel, the CSR pair
and the counting plan, walked item by item in plain loops by a test harness
(tests/native/plan_emul.cpp) and compared with the oracle."""

import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import vp_counts
from synth import chung_lu_graph, config_graph, uniform_graph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_21848_amd", "csrc")


@pytest.fixture(scope="module")
def emul_lib(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("emul") / "plan_emul.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", so,
                           os.path.join(ROOT, "tests", "native", "plan_emul.cpp"),
                           os.path.join(ROOT, "tests", "native", "host_build.cpp"), os.path.join(CSRC, "plan.cpp")])
    lib = ctypes.CDLL(so)
    u64 = ctypes.c_uint64
    lib.plan_check_sizes.argtypes = [u64, u64, u64, u64]
    lib.plan_check_sizes.restype = ctypes.c_int
    return lib


@pytest.fixture(scope="module")
def emul(emul_lib):
    lib = emul_lib
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.plan_emulate.argtypes = [i32, i32, i64, p, p, p, i32, i32, i32, i32, i32, p]

    def run(g, T=-1, L=-1, sw=-1, pw=-1, R=-1):
        out = np.zeros(13, np.int64)
        if R < 0 and L >= 0:
            R = min(L, 4096)
        rc = lib.plan_emulate(g.n_u, g.n_v, g.m, g.u.ctypes.data, g.v.ctypes.data,
                              g.sign.ctypes.data, T, L, R, sw, pw, out.ctypes.data)
        assert rc == 0, rc
        return out
    return run


# (hub_T, window_L, small_work, part_work, reverse_L)
CONFIGS = [(0, 256, 2, 4096, 64), (128, 256, 64, 4096, 256), (256, 512, 512, 8192, 128),
           (0, 32768, 512, 1 << 20, 4096), (256, 1024, 16, 4096, 512), (0, 2048, 512, 4096, 2048),
           (128, 1024, 300, 4096, 1024)]


def _check(o, r):
    assert (o[0], o[1], o[2]) == (r.balanced, r.unbalanced, r.total)
    assert o[3] == r.wedges                      # closed-form W_VP of the library
    assert o[4] + o[5] + o[6] == o[3]            # sparse + skipped + dense = W_VP
    assert o[7] == o[4]                          # every planned wedge walked once


@pytest.mark.parametrize("seed", range(12))
def test_plan_partition_matches_oracle(emul, seed):
    rng = np.random.default_rng(seed)
    g = chung_lu_graph(int(rng.integers(300, 3000)), int(rng.integers(300, 3000)),
                       int(rng.integers(1000, 30000)), 2.0, 1.9, 0.4, seed=seed)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    for cfg in CONFIGS:
        _check(emul(g, *cfg), r)


def test_plan_on_tiny_workload(emul):
    g = config_graph("tiny")
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    for cfg in CONFIGS:
        _check(emul(g, *cfg), r)


def test_plan_on_small_and_degenerate_graphs(emul):
    for seed in range(40):
        rng = np.random.default_rng(1000 + seed)
        n_u, n_v = int(rng.integers(1, 20)), int(rng.integers(1, 20))
        g = uniform_graph(n_u, n_v, int(rng.integers(0, n_u * n_v + 1)), 0.5, seed=seed)
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
        for cfg in [(0, 256, 2, 4096, 64), (0, 256, 512, 4096, 128)]:
            _check(emul(g, *cfg), r)


def test_hub_block_on_dense_graph(emul):
    # a dense graph where the hub block covers most pairs
    g = chung_lu_graph(600, 500, 60000, 2.5, 2.5, 0.3, seed=7)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    for cfg in [(256, 256, 64, 4096, 64), (384, 512, 2, 4096, 512), (0, 512, 512, 4096, 128)]:
        o = emul(g, *cfg)
        _check(o, r)
    assert emul(g, 256, 256, 64, 4096, 128)[6] > 0


def test_reverse_items_split_into_parts(emul):
    # every vertex below a 256 window has about 250-300 neighbours, so reverse
    # items exceed 255 segments and are split into parts
    g = chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    for cfg in [(0, 256, 512, 1 << 20, 64), (0, 256, 2, 4096, 256), (128, 256, 64, 4096, 128)]:
        o = emul(g, *cfg)
        _check(o, r)
        assert o[11] > 0  # multi-part reduces exist


@pytest.fixture(scope="module")
def emul_pv(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("emulpv") / "plan_emul.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", so,
                           os.path.join(ROOT, "tests", "native", "plan_emul.cpp"),
                           os.path.join(ROOT, "tests", "native", "host_build.cpp"), os.path.join(CSRC, "plan.cpp")])
    lib = ctypes.CDLL(so)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.plan_emulate_pv.argtypes = [i32, i32, i64, p, p, p, i32, i32, i32, i32, p, p, p, p, p]

    def run(g, L=-1, R=-1, sw=-1, edges=False, T=0):
        n = g.n_u + g.n_v
        bal = np.zeros(n, np.int64)
        unb = np.zeros(n, np.int64)
        be = np.zeros(g.m, np.int64) if edges else None
        ue = np.zeros(g.m, np.int64) if edges else None
        out = np.zeros(5, np.int64)
        if R < 0 and L >= 0:
            R = min(L, 4096)
        rc = lib.plan_emulate_pv(g.n_u, g.n_v, g.m, g.u.ctypes.data, g.v.ctypes.data,
                                 g.sign.ctypes.data, T, L, R, sw, bal.ctypes.data, unb.ctypes.data,
                                 None if be is None else be.ctypes.data,
                                 None if ue is None else ue.ctypes.data, out.ctypes.data)
        assert rc == 0, rc
        if edges:
            return out, bal, unb, be, ue
        return out, bal, unb
    return run


@pytest.mark.parametrize("seed", range(6))
def test_per_vertex_plan_matches_oracle(emul_pv, seed):
    rng = np.random.default_rng(50 + seed)
    g = chung_lu_graph(int(rng.integers(300, 2500)), int(rng.integers(300, 2500)),
                       int(rng.integers(1000, 30000)), 2.0, 1.9, 0.4, seed=seed)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True)
    want_bal = np.concatenate([r.bal_u, r.bal_v])
    want_unb = np.concatenate([r.unb_u, r.unb_v])
    for L, R, sw in [(-1, -1, -1), (256, 64, 2), (512, 512, 64), (1024, 128, 512)]:
        out, bal, unb = emul_pv(g, L, R, sw)
        assert (out[0], out[1], out[2]) == (r.balanced, r.unbalanced, r.total)
        assert np.array_equal(bal, want_bal), (L, R, sw)
        assert np.array_equal(unb, want_unb), (L, R, sw)


def test_per_vertex_plan_dense_graph(emul_pv):
    # reverse endpoints with more than 255 runs become direct items, and
    # pivots with wide windows are split into key windows
    g = chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True)
    for L, R in [(256, 64), (512, 256), (-1, -1)]:
        out, bal, unb = emul_pv(g, L, R)
        assert np.array_equal(bal, np.concatenate([r.bal_u, r.bal_v]))
        assert np.array_equal(unb, np.concatenate([r.unb_u, r.unb_v]))


def test_per_vertex_plan_key_windows(emul_pv):
    # sides wider than one key window: direct items split into windows
    g = chung_lu_graph(20000, 12000, 120000, 2.1, 1.9, 0.4, seed=4)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True)
    out, bal, unb = emul_pv(g)
    assert (out[0], out[1], out[2]) == (r.balanced, r.unbalanced, r.total)
    assert np.array_equal(bal, np.concatenate([r.bal_u, r.bal_v]))
    assert np.array_equal(unb, np.concatenate([r.unb_u, r.unb_v]))


@pytest.mark.parametrize("seed", range(4))
def test_per_edge_plan_matches_oracle(emul_pv, seed):
    # every wedge of the per-vertex plan credits its run's first edge and its
    # walked entry's edge, found through the positions the plan records
    rng = np.random.default_rng(90 + seed)
    g = chung_lu_graph(int(rng.integers(300, 2500)), int(rng.integers(300, 2500)),
                       int(rng.integers(1000, 30000)), 2.0, 1.9, 0.4, seed=seed)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_edge=True)
    for L, R, sw in [(-1, -1, -1), (256, 64, 2), (1024, 128, 512)]:
        out, _, _, be, ue = emul_pv(g, L, R, sw, edges=True)
        assert np.array_equal(be, r.bal_e), (L, R, sw)
        assert np.array_equal(ue, r.unb_e), (L, R, sw)


def test_per_edge_plan_dense_graph(emul_pv):
    g = chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_edge=True)
    for L, R in [(256, 64), (-1, -1)]:
        out, _, _, be, ue = emul_pv(g, L, R, edges=True)
        assert np.array_equal(be, r.bal_e) and np.array_equal(ue, r.unb_e)


def test_plan_size_guard(emul_lib):
    """Plans whose run indices or item counts would not fit their 32-bit
    fields are refused with DBBC_E_TOO_LARGE (-7) instead of wrapping."""
    f = emul_lib.plan_check_sizes
    u32, i32 = (1 << 32) - 1, (1 << 31) - 1
    assert f(u32, i32, i32, i32) == 0
    assert f(u32 + 1, 0, 0, 0) == -7
    assert f(0, i32 + 1, 0, 0) == -7
    assert f(0, 0, i32 + 1, 0) == -7
    assert f(0, 0, 0, i32 + 1) == -7
    assert f(0, 0, 0, 0) == 0


@pytest.mark.parametrize("seed", range(4))
def test_per_vertex_plan_with_dense_block(emul_pv, seed):
    """Per-vertex and per-edge plans with a dense block: hub runs, completed
    hub-pair counts, block-wedge credits and the hub items' walks give the
    oracle's counts."""
    rng = np.random.default_rng(130 + seed)
    g = chung_lu_graph(int(rng.integers(600, 2500)), int(rng.integers(600, 2500)),
                       int(rng.integers(8000, 40000)), 2.0, 1.9, 0.4, seed=seed)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True, per_edge=True)
    for T, L, R, sw in [(128, -1, -1, -1), (256, 256, 64, 2), (128, 512, 512, 64), (256, 1024, 128, 512)]:
        out, bal, unb, be, ue = emul_pv(g, L, R, sw, edges=True, T=T)
        assert out[4] == T
        assert (out[0], out[1], out[2]) == (r.balanced, r.unbalanced, r.total), (T, L, R, sw)
        assert np.array_equal(bal, np.concatenate([r.bal_u, r.bal_v])), (T, L, R, sw)
        assert np.array_equal(unb, np.concatenate([r.unb_u, r.unb_v])), (T, L, R, sw)
        assert np.array_equal(be, r.bal_e) and np.array_equal(ue, r.unb_e), (T, L, R, sw)


def test_per_vertex_plan_dense_block_on_dense_graph(emul_pv):
    g = chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True, per_edge=True)
    for T, L, R in [(128, 256, 64), (256, 512, 256), (256, -1, -1)]:
        out, bal, unb, be, ue = emul_pv(g, L, R, edges=True, T=T)
        assert np.array_equal(bal, np.concatenate([r.bal_u, r.bal_v]))
        assert np.array_equal(unb, np.concatenate([r.unb_u, r.unb_v]))
        assert np.array_equal(be, r.bal_e) and np.array_equal(ue, r.unb_e)
