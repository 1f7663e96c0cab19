"""GPU: the device planner against the host planner and the oracle.

Plans are made on the device by default (kernels and scans over the CSR
entries); DBBC_OPT_HOST_PLAN makes them with the host planner.  Both split
the same vertex-priority wedges (Algorithm 1, with each pivot's work sized as
in Eq. 1) into the same classes of work items, so per counting kernel the
wedges and the CSR runs handed to it must be equal, and both counts must equal
the oracle's.  The grouping of small items and the parts of heavy items may
differ between the planners; the item counts are therefore not compared.
Per-vertex and per-edge plans (tagged runs, key windows, the hub pivots'
tally items, the dense block's credit constants) are checked through their
results: every vertex's and every edge's counts from both planners equal the
oracle's.
"""

import numpy as np
import pytest

from oracle import vp_counts
from synth import chung_lu_graph, uniform_graph

pytestmark = pytest.mark.gpu

KERNELS = ("direct", "reverse", "small", "hash")

# (window_L, reverse_L, hub_T, small_work, part_work); -1 = default
OPTS = [
    {},
    dict(window_L=256, reverse_L=64, small_work=2, part_work=4096),
    dict(window_L=512, reverse_L=128, small_work=64, part_work=4096),
    dict(window_L=256, reverse_L=256, hub_T=128),
    dict(hub_T=0, part_work=4096),
    dict(window_L=1024, reverse_L=64, hub_T=256, small_work=512),
    dict(window_L=256, reverse_L=64, hub_T=256, small_work=300, part_work=5000),
]


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


def _timed(dbbc, h, flags=0, **opts):
    c = h.count(flags=flags | dbbc.DBBC_OPT_TIME_KERNELS, **opts)
    recs = dbbc.dbbc_last_kernel_times(h.handle)
    per = {r["name"]: (r["wedges"], r["segments"]) for r in recs if r["name"] in KERNELS}
    reduces = sum(r["items"] for r in recs if r["name"] == "reduce")
    return (c.balanced, c.unbalanced, c.total, c.wedges), per, reduces


def _planted_reverse_parts():
    """64 hubs joined to all 3,000 V vertices, and 400 U vertices of degree
    150: with window_L = 256 and reverse_L = 64, the 208 of the latter ranked
    past the window are reverse endpoints with 150 runs each (one per mid,
    every mid's row starting with the 64 hubs), so their reverse items are cut
    into parts of at most 127 runs."""
    rng = np.random.default_rng(11)
    n_hub, n_wide, n_v = 64, 400, 3000
    us, vs = [], []
    for x in range(n_hub):
        us.append(np.full(n_v, x, np.int32))
        vs.append(np.arange(n_v, dtype=np.int32))
    for k in range(n_wide):
        us.append(np.full(150, n_hub + k, np.int32))
        vs.append(rng.choice(n_v, 150, replace=False).astype(np.int32))
    u = np.concatenate(us)
    v = np.concatenate(vs)
    s = np.where(rng.random(len(u)) < 0.4, -1, 1).astype(np.int8)
    return n_hub + n_wide, n_v, u, v, s


def _as_tuple(g):
    return g.n_u, g.n_v, g.u, g.v, g.sign


def test_planners_agree(dbbc):
    graphs = [
        ("chung_lu_3k", _as_tuple(chung_lu_graph(3000, 2500, 60000, 2.0, 1.9, 0.4, seed=5))),
        ("chung_lu_9k", _as_tuple(chung_lu_graph(9000, 8000, 200000, 2.0, 1.9, 0.4, seed=41))),
        ("uniform_300", _as_tuple(uniform_graph(300, 300, 20000, 0.5, seed=3))),
        ("planted_reverse_parts", _planted_reverse_parts()),
    ]
    for name, (n_u, n_v, u, v, s) in graphs:
        r = vp_counts(n_u, n_v, u, v, s)
        want = (r.balanced, r.unbalanced, r.total, r.wedges)
        with dbbc.Graph(n_u, n_v, u, v, s) as h:
            for opts in OPTS:
                _say("planners", name, opts)
                got_d, per_d, _ = _timed(dbbc, h, **opts)
                got_h, per_h, _ = _timed(dbbc, h, flags=dbbc.DBBC_OPT_HOST_PLAN, **opts)
                assert got_d == want, (name, opts)
                assert got_h == want, (name, opts)
                assert per_d == per_h, (name, opts, per_d, per_h)


def test_planted_graph_has_reverse_parts(dbbc):
    # the planted graph reaches the reverse parts and their reduces: the
    # forced configuration has more reduces than direct parts alone give
    n_u, n_v, u, v, s = _planted_reverse_parts()
    with dbbc.Graph(n_u, n_v, u, v, s) as h:
        _, _, red_small_window = _timed(dbbc, h, window_L=256, reverse_L=64, part_work=1 << 30)
        assert red_small_window >= 208
        r = vp_counts(n_u, n_v, u, v, s)
        c = h.count(window_L=256, reverse_L=64, part_work=1 << 30)
        assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total)


def test_empty_and_tiny_graphs(dbbc):
    cases = [(1, 1, [], [], []), (2, 3, [0], [2], [-1]), (3, 3, [0, 0, 1, 1], [0, 1, 0, 1], [1, -1, -1, 1])]
    for n_u, n_v, u, v, s in cases:
        u = np.asarray(u, np.int32)
        v = np.asarray(v, np.int32)
        s = np.asarray(s, np.int8)
        r = vp_counts(n_u, n_v, u, v, s)
        with dbbc.Graph(n_u, n_v, u, v, s) as h:
            for flags in (0, dbbc.DBBC_OPT_HOST_PLAN):
                c = h.count(flags=flags)
                assert (c.balanced, c.unbalanced, c.total, c.wedges) == (r.balanced, r.unbalanced, r.total,
                                                                         r.wedges)


def test_planners_agree_at_full_size(dbbc):
    # the 50M-edge workload: both planners' counts equal the oracle's cached
    # counts, and every counting kernel gets the same wedges and runs
    import json
    import os

    from golden_io import GOLDEN
    from synth import config_graph
    with open(os.path.join(GOLDEN, "oracle_cache.json")) as f:
        cache = json.load(f)["skewed50m"]
    g = config_graph("skewed50m")
    want = (cache["balanced"], cache["unbalanced"], cache["total"], cache["wedges"])
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        for opts in ({}, dict(window_L=8192, reverse_L=1024, part_work=1 << 20)):
            _say("planners at full size", opts)
            got_d, per_d, _ = _timed(dbbc, h, **opts)
            got_h, per_h, _ = _timed(dbbc, h, flags=dbbc.DBBC_OPT_HOST_PLAN, **opts)
            assert got_d == want and got_h == want, opts
            assert per_d == per_h, (opts, per_d, per_h)


WIDE = 0x2  # DBBC_OPT_WIDE_EDGES


def test_per_vertex_and_per_edge_planners_agree(dbbc):
    graphs = [
        ("chung_lu_3k", _as_tuple(chung_lu_graph(3000, 2500, 60000, 2.0, 1.9, 0.4, seed=5)),
         ({}, dict(window_L=256, reverse_L=64, small_work=2), dict(hub_T=256, window_L=512, reverse_L=128))),
        ("planted_reverse_parts", _planted_reverse_parts(),
         (dict(window_L=256, reverse_L=64), dict(hub_T=128, window_L=256, reverse_L=64))),
        ("dense", _as_tuple(chung_lu_graph(1200, 1000, 300000, 3.0, 3.0, 0.45, seed=9)),
         (dict(hub_T=512), dict(hub_T=1024, window_L=1024, reverse_L=256), dict(hub_T=0, window_L=256))),
    ]
    for name, (n_u, n_v, u, v, s), opts_list in graphs:
        r = vp_counts(n_u, n_v, u, v, s, per_vertex=True, per_edge=True)
        with dbbc.Graph(n_u, n_v, u, v, s) as h:
            for opts in opts_list:
                for flags in (0, dbbc.DBBC_OPT_HOST_PLAN):
                    _say("per-vertex planners", name, opts, flags)
                    c, bu, bv, uu, uv = h.count_per_vertex(flags=flags, **opts)
                    assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total)
                    for t, want in ((bu, r.bal_u), (bv, r.bal_v), (uu, r.unb_u), (uv, r.unb_v)):
                        assert np.array_equal(t.cpu().numpy(), want), (name, opts, flags)
                    for f in (flags, flags | WIDE):
                        c, be, ue = h.count_per_edge(flags=f, **opts)
                        assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total)
                        assert np.array_equal(be.cpu().numpy(), r.bal_e), (name, opts, f)
                        assert np.array_equal(ue.cpu().numpy(), r.unb_e), (name, opts, f)


def test_per_vertex_empty_and_tiny_graphs(dbbc):
    cases = [(1, 1, [], [], []), (2, 3, [0], [2], [-1]), (3, 3, [0, 0, 1, 1], [0, 1, 0, 1], [1, -1, -1, 1])]
    for n_u, n_v, u, v, s in cases:
        u = np.asarray(u, np.int32)
        v = np.asarray(v, np.int32)
        s = np.asarray(s, np.int8)
        r = vp_counts(n_u, n_v, u, v, s, per_vertex=True, per_edge=True)
        with dbbc.Graph(n_u, n_v, u, v, s) as h:
            for flags in (0, dbbc.DBBC_OPT_HOST_PLAN):
                _, bu, bv, uu, uv = h.count_per_vertex(flags=flags)
                for t, want in ((bu, r.bal_u), (bv, r.bal_v), (uu, r.unb_u), (uv, r.unb_v)):
                    assert np.array_equal(t.cpu().numpy(), want), (n_u, n_v, flags)
                _, be, ue = h.count_per_edge(flags=flags)
                assert np.array_equal(be.cpu().numpy(), r.bal_e) and np.array_equal(ue.cpu().numpy(), r.unb_e)
