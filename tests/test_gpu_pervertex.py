"""GPU parity of the per-vertex pass (dbbc_count_per_vertex): for every
vertex, the balanced and unbalanced butterflies containing it, bit-exact
against the oracle (and against the paper's printed values on its figure),
plus the invariant that each side's entries sum to twice the global counts;
at the largest size every vertex against digests of the oracle's arrays."""

import json
import os

import numpy as np
import pytest

from oracle import brute_per_vertex, vp_counts
from synth import chung_lu_graph, config_graph, uniform_graph

from golden_io import GOLDEN, load

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dbbc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2609_21848_amd as mod
    mod.load()  # raises if the HIP library is missing
    return mod


def _say(*a):
    print(*a, flush=True)


def _digest(a) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def _pv(dbbc, n_u, n_v, u, v, s, **opts):
    with dbbc.Graph(n_u, n_v, u, v, s) as h:
        c, bu, bv, uu, uv = h.count_per_vertex(**opts)
        return c, bu.cpu().numpy(), bv.cpu().numpy(), uu.cpu().numpy(), uv.cpu().numpy()


def _check(dbbc, g, opts_list=({},)):
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True)
    for opts in opts_list:
        c, bu, bv, uu, uv = _pv(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign, **opts)
        assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total), opts
        assert np.array_equal(bu, r.bal_u), opts
        assert np.array_equal(bv, r.bal_v), opts
        assert np.array_equal(uu, r.unb_u), opts
        assert np.array_equal(uv, r.unb_v), opts


def test_paper_figure_vertex_values(dbbc):
    (fx,) = load("fig_comparison.txt")
    n_u, n_v, u, v, s = fx.arrays()
    c, bu, bv, uu, uv = _pv(dbbc, n_u, n_v, u, v, s)
    for e in fx.expect:
        if e[0] == "vertex_balanced":
            idx = fx.vertex(e[1])
            got = bu[idx] if idx < n_u else bv[idx - n_u]
            assert got == int(e[2]), e
    assert bu.sum() == 2 * c.balanced and bv.sum() == 2 * c.balanced


def test_tiny_graphs_against_brute_force(dbbc):
    for seed in range(30):
        rng = np.random.default_rng(700 + seed)
        n_u, n_v = int(rng.integers(1, 14)), int(rng.integers(1, 14))
        g = uniform_graph(n_u, n_v, int(rng.integers(0, n_u * n_v + 1)), float(rng.random()), seed=seed)
        bu, bv, uu, uv = brute_per_vertex(g.n_u, g.n_v, g.u, g.v, g.sign)
        _say("tiny pv", seed, n_u, n_v, g.m)
        c, gbu, gbv, guu, guv = _pv(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign)
        assert np.array_equal(gbu, bu) and np.array_equal(gbv, bv)
        assert np.array_equal(guu, uu) and np.array_equal(guv, uv)


def test_random_graphs_and_options(dbbc):
    for seed in range(8):
        rng = np.random.default_rng(800 + seed)
        g = chung_lu_graph(int(rng.integers(100, 3000)), int(rng.integers(100, 3000)),
                           int(rng.integers(500, 30000)), 2.0, 1.9, 0.4, seed=seed)
        _say("random pv", seed, g.n_u, g.n_v, g.m)
        _check(dbbc, g, ({}, {"window_L": 256, "reverse_L": 64, "small_work": 2},
                         {"window_L": 512, "long_len": 16}, {"long_len": 65536, "small_work": 64}))


def test_dense_graph_reverse_items_as_direct(dbbc):
    # reverse endpoints with more than 255 runs are counted as direct items
    g = chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9)
    _say("dense pv")
    _check(dbbc, g, ({"window_L": 256, "reverse_L": 64}, {"window_L": 256, "reverse_L": 256}, {}))


def test_tiny_workload_and_key_windows(dbbc):
    _check(dbbc, config_graph("tiny"), ({}, {"window_L": 256}))
    # sides wider than one key window of the direct items
    g = chung_lu_graph(20000, 12000, 120000, 2.1, 1.9, 0.4, seed=4)
    _check(dbbc, g)


def test_powerlaw2m_full_size(dbbc):
    g = config_graph("powerlaw2m")
    _say("powerlaw2m pv")
    _check(dbbc, g)


def test_skewed50m_invariants(dbbc):
    with open(os.path.join(GOLDEN, "oracle_cache.json")) as f:
        cache = json.load(f)["skewed50m"]
    g = config_graph("skewed50m")
    _say("skewed50m pv")
    c, bu, bv, uu, uv = _pv(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign)
    assert (c.balanced, c.unbalanced, c.total) == (cache["balanced"], cache["unbalanced"],
                                                   cache["total"])
    for arr, want in ((bu, c.balanced), (bv, c.balanced), (uu, c.unbalanced), (uv, c.unbalanced)):
        assert (arr >= 0).all()
        assert int(arr.sum()) == 2 * want
    # every vertex against the oracle: SHA-256 of the oracle's arrays,
    # written by tests/golden/make_oracle_cache.py --local
    digests = cache["local"]["sha256"]
    for name, arr in (("bal_u", bu), ("bal_v", bv), ("unb_u", uu), ("unb_v", uv)):
        assert _digest(arr) == digests[name], f"{name} differs from the oracle's"


def test_dense_block_sweep(dbbc):
    """The dense block in the per-vertex pass: hub_T in {0, 128, ..., 4096},
    every vertex against the oracle (the hub pairs' counts completed by the
    block's products, their credits and the hub mids' credits computed by
    the credit products, the rest by the sparse kernels)."""
    g = chung_lu_graph(9000, 8000, 200000, 2.0, 1.9, 0.4, seed=41)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        for opts in ({"hub_T": 0}, {"hub_T": 128}, {"hub_T": 384}, {"hub_T": 1024},
                     {"hub_T": 2048, "window_L": 2048, "reverse_L": 512}, {"hub_T": 4096},
                     {"hub_T": 256, "window_L": 256, "reverse_L": 64, "small_work": 2}):
            _say("dense-block pv", opts)
            c, bu, bv, uu, uv = h.count_per_vertex(**opts)
            assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total), opts
            for t, want in ((bu, r.bal_u), (bv, r.bal_v), (uu, r.unb_u), (uv, r.unb_v)):
                assert np.array_equal(t.cpu().numpy(), want), opts


def test_dense_block_on_dense_graph(dbbc):
    g = chung_lu_graph(1200, 1000, 300000, 3.0, 3.0, 0.45, seed=9)
    _say("dense-block pv dense graph")
    _check(dbbc, g, ({"hub_T": 512}, {"hub_T": 1024, "window_L": 1024, "reverse_L": 256}))
