"""GPU parity of the per-edge pass (dbbc_count_per_edge): for every input
record, the balanced and unbalanced butterflies containing its edge,
bit-exact against the oracle (and the paper's printed values on its
figure); at the largest size, every edge against digests of the oracle's
arrays, stored values at the highest-degree vertices, sampled edges against
the oracle's local count and the invariants that tie the edge counts to the
global and the per-vertex counts."""

import json
import os

import numpy as np
import pytest

from oracle import brute_per_edge, edge_counts_at, vp_counts
from synth import chung_lu_graph, config_graph, uniform_graph

from golden_io import GOLDEN, load

pytestmark = pytest.mark.gpu

WIDE = 0x2  # DBBC_OPT_WIDE_EDGES: every edge's credits in two words


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


def _pe(dbbc, n_u, n_v, u, v, s, **opts):
    with dbbc.Graph(n_u, n_v, u, v, s) as h:
        c, be, ue = h.count_per_edge(**opts)
        return c, be.cpu().numpy(), ue.cpu().numpy()


def _check(dbbc, g, opts_list=({},)):
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_edge=True)
    for opts in opts_list:
        c, be, ue = _pe(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign, **opts)
        assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total), opts
        assert np.array_equal(be, r.bal_e), opts
        assert np.array_equal(ue, r.unb_e), opts


def test_paper_figure_edge_values(dbbc):
    (fx,) = load("fig_comparison.txt")
    n_u, n_v, u, v, s = fx.arrays()
    c, be, ue = _pe(dbbc, n_u, n_v, u, v, s)
    edge_index = {(a, b): i for i, (a, b, _) in enumerate(fx.edges)}
    for e in fx.expect:
        if e[0] == "edge_balanced":
            assert be[edge_index[(fx.left[e[1]], fx.right[e[2]])]] == int(e[3]), e
    assert be.sum() == 4 * c.balanced and (ue == 0).all()


def test_tiny_graphs_against_brute_force(dbbc):
    for seed in range(30):
        rng = np.random.default_rng(900 + seed)
        n_u, n_v = int(rng.integers(1, 14)), int(rng.integers(1, 14))
        g = uniform_graph(n_u, n_v, int(rng.integers(0, n_u * n_v + 1)), float(rng.random()), seed=seed)
        bb, bu = brute_per_edge(g.n_u, g.n_v, g.u, g.v, g.sign)
        _say("tiny pe", seed, n_u, n_v, g.m)
        for opts in ({}, {"flags": WIDE}):
            c, be, ue = _pe(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign, **opts)
            assert list(be) == bb and list(ue) == bu, opts


def test_duplicate_records(dbbc):
    # the last record of a repeated pair carries the edge; earlier ones read 0
    g = chung_lu_graph(400, 300, 4000, 2.0, 1.9, 0.4, seed=21)
    rng = np.random.default_rng(21)
    rep = rng.choice(g.m, 300, replace=False)
    u = np.concatenate([g.u[rep], g.u]).astype(np.int32)
    v = np.concatenate([g.v[rep], g.v]).astype(np.int32)
    s = np.concatenate([-g.sign[rep], g.sign]).astype(np.int8)  # overwritten by the later record
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_edge=True)
    c, be, ue = _pe(dbbc, g.n_u, g.n_v, u, v, s)
    assert (c.balanced, c.unbalanced) == (r.balanced, r.unbalanced)
    assert (be[:300] == 0).all() and (ue[:300] == 0).all()
    assert np.array_equal(be[300:], r.bal_e) and np.array_equal(ue[300:], r.unb_e)


def test_random_graphs_and_options(dbbc):
    for seed in range(8):
        rng = np.random.default_rng(1800 + seed)
        g = chung_lu_graph(int(rng.integers(100, 3000)), int(rng.integers(100, 3000)),
                           int(rng.integers(500, 30000)), 2.0, 1.9, 0.4, seed=seed)
        _say("random pe", seed, g.n_u, g.n_v, g.m)
        _check(dbbc, g, ({}, {"window_L": 256, "reverse_L": 64, "small_work": 2},
                         {"window_L": 512, "long_len": 16}, {"long_len": 65536, "small_work": 64},
                         {"flags": WIDE}, {"window_L": 256, "reverse_L": 64, "small_work": 2,
                                           "flags": WIDE}))


def test_dense_graph_reverse_items_as_direct(dbbc):
    g = chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9)
    _say("dense pe")
    _check(dbbc, g, ({"window_L": 256, "reverse_L": 64}, {}, {"flags": WIDE}))


def test_tiny_workload_key_windows_and_repeat(dbbc):
    _check(dbbc, config_graph("tiny"), ({}, {"window_L": 256}))
    g = chung_lu_graph(20000, 12000, 120000, 2.1, 1.9, 0.4, seed=4)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_edge=True)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        # per-vertex first (plan made without the edge buffers), then twice per edge
        h.count_per_vertex()
        for _ in range(2):
            c, be, ue = h.count_per_edge()
            assert np.array_equal(be.cpu().numpy(), r.bal_e)
            assert np.array_equal(ue.cpu().numpy(), r.unb_e)


def test_powerlaw2m_full_size(dbbc):
    g = config_graph("powerlaw2m")
    _say("powerlaw2m pe")
    _check(dbbc, g)


def test_skewed50m_samples_and_invariants(dbbc):
    import torch
    with open(os.path.join(GOLDEN, "oracle_cache.json")) as f:
        cache = json.load(f)["skewed50m"]
    g = config_graph("skewed50m")
    _say("skewed50m pe")
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        c, be, ue = h.count_per_edge()
        assert (c.balanced, c.unbalanced, c.total) == (cache["balanced"], cache["unbalanced"],
                                                       cache["total"])
        _, bu, bv, uu, uv = h.count_per_vertex()
        assert int(be.sum()) == 4 * c.balanced and int(ue.sum()) == 4 * c.unbalanced
        assert bool((be >= 0).all()) and bool((ue >= 0).all())
        # the edges at a vertex hold two places of each of its butterflies
        dev = be.device
        for e_arr, pu, pv in ((be, bu, bv), (ue, uu, uv)):
            su = torch.zeros(g.n_u, dtype=torch.int64, device=dev)
            su.index_add_(0, torch.from_numpy(g.u.astype(np.int64)).to(dev), e_arr)
            sv = torch.zeros(g.n_v, dtype=torch.int64, device=dev)
            sv.index_add_(0, torch.from_numpy(g.v.astype(np.int64)).to(dev), e_arr)
            assert torch.equal(su, 2 * pu) and torch.equal(sv, 2 * pv)
        be, ue = be.cpu().numpy(), ue.cpu().numpy()
    # every edge against the oracle: SHA-256 of the oracle's arrays and the
    # explicit values of edges at the highest-degree vertices (those whose
    # runs keep two-word credits), written by make_oracle_cache.py --local
    local = cache["local"]
    assert _digest(be) == local["sha256"]["bal_e"], "balanced per-edge counts differ from the oracle's"
    assert _digest(ue) == local["sha256"]["unb_e"], "unbalanced per-edge counts differ from the oracle's"
    edges = np.array(local["edges"], np.int64)
    assert list(be[edges]) == local["bal_e"] and list(ue[edges]) == local["unb_e"]
    # sampled edges against the oracle's count around each edge
    deg_u = np.bincount(g.u, minlength=g.n_u)
    deg_v = np.bincount(g.v, minlength=g.n_v)
    cost = deg_u[g.u].astype(np.int64) * deg_v[g.v]
    rng = np.random.default_rng(5)
    cheap = np.flatnonzero(cost <= 2_000_000)
    mid = np.flatnonzero((cost > 2_000_000) & (cost <= 20_000_000))
    some = np.concatenate([rng.choice(cheap, 200, replace=False), rng.choice(mid, 10, replace=False)])
    _say("skewed50m pe: sampled edges against the oracle")
    lb, lu = edge_counts_at(g.n_u, g.n_v, g.u, g.v, g.sign, some)
    assert list(be[some]) == lb and list(ue[some]) == lu


def test_crossing_hubs_packed_and_wide_credits(dbbc):
    """Two hubs of degree 70,000, one per side, over random edges: runs whose
    mid is a hub have mid degree x the keys' side's largest degree >= 2^32,
    so the planner gives them two-word credits, while every other run packs
    both credits into one word.  Both forms in one plan, every edge and
    vertex against the oracle."""
    n_u = n_v = 70000
    base = chung_lu_graph(n_u, n_v, 200000, 2.1, 2.1, 0.4, seed=21)
    rng = np.random.default_rng(21)
    hu, hv = 17, 23
    u = np.concatenate([base.u, np.full(n_v, hu, np.int32), np.arange(n_u, dtype=np.int32)])
    v = np.concatenate([base.v, np.arange(n_v, dtype=np.int32), np.full(n_u, hv, np.int32)])
    _, first = np.unique(u.astype(np.int64) * n_v + v, return_index=True)
    first = np.sort(first)
    u, v = u[first], v[first]
    s = np.where(rng.random(u.shape[0]) < 0.4, -1, 1).astype(np.int8)
    deg_u = np.bincount(u, minlength=n_u)
    deg_v = np.bincount(v, minlength=n_v)
    assert int(deg_u[hu]) * int(deg_v.max()) >= 1 << 32 and int(deg_v[hv]) * int(deg_u.max()) >= 1 << 32
    _say("crossing hubs pe", n_u, n_v, u.shape[0])
    r = vp_counts(n_u, n_v, u, v, s, per_vertex=True, per_edge=True)
    with dbbc.Graph(n_u, n_v, u, v, s) as h:
        # without and with a dense block (which holds both hubs: pair counts
        # of three 7-bit digits in its products; the hubs' rows keep their
        # edge credits in two words, its other rows in one packed word, and
        # with the wide-edges option every row in two words)
        for opts in ({"hub_T": 0}, {"hub_T": 256}, {"hub_T": 256, "flags": WIDE}):
            c, be, ue = h.count_per_edge(**opts)
            assert (c.balanced, c.unbalanced, c.total, c.wedges) == (r.balanced, r.unbalanced, r.total,
                                                                     r.wedges)
            assert np.array_equal(be.cpu().numpy(), r.bal_e), opts
            assert np.array_equal(ue.cpu().numpy(), r.unb_e), opts
            if "flags" in opts:
                continue
            _, bu, bv, uu, uv = h.count_per_vertex(**opts)
            for t, want in ((bu, r.bal_u), (bv, r.bal_v), (uu, r.unb_u), (uv, r.unb_v)):
                assert np.array_equal(t.cpu().numpy(), want), opts


def test_dense_block_sweep(dbbc):
    """The dense block in the per-edge pass: hub_T in {0, 128, ..., 4096},
    every edge against the oracle (the block's edges take their pivot-mid
    and end-mid credits from the credit products)."""
    g = chung_lu_graph(9000, 8000, 200000, 2.0, 1.9, 0.4, seed=41)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_edge=True)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        for opts in ({"hub_T": 0}, {"hub_T": 128}, {"hub_T": 384}, {"hub_T": 1024},
                     {"hub_T": 2048, "window_L": 2048, "reverse_L": 512}, {"hub_T": 4096},
                     {"hub_T": 256, "flags": WIDE}):
            _say("dense-block pe", opts)
            c, be, ue = h.count_per_edge(**opts)
            assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total), opts
            assert np.array_equal(be.cpu().numpy(), r.bal_e), opts
            assert np.array_equal(ue.cpu().numpy(), r.unb_e), opts


def test_dense_block_on_dense_graph(dbbc):
    g = chung_lu_graph(1200, 1000, 300000, 3.0, 3.0, 0.45, seed=9)
    _say("dense-block pe dense graph")
    _check(dbbc, g, ({"hub_T": 512}, {"hub_T": 1024, "window_L": 1024, "reverse_L": 256}))
