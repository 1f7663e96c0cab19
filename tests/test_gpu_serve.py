"""GPU checks of the request server (dbbc_server_*): continuous batching of
count requests over resident graphs of mixed sizes.  Every result must equal
the count of the same graph alone (dbbc_count) and the oracle's, whatever
launch it landed in; admission by HBM footprint rejects or evicts uploads."""

import numpy as np
import pytest

from oracle import vp_counts
from synth import batch_graph, chung_lu_graph, pool_graph

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


def _want(g):
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    return (r.balanced, r.unbalanced, r.total, r.wedges)


def _pool():
    gs = [pool_graph(i) for i in range(0, 1000, 40) if pool_graph(i).m <= 400_000]
    gs += [batch_graph(i) for i in range(0, 4096, 300)]
    gs.append(chung_lu_graph(1500, 1200, 150000, 2.4, 2.2, 0.35, seed=3))
    return gs


def test_served_results_equal_alone_and_oracle(dbbc):
    gs = _pool()
    want = [_want(g) for g in gs]
    # alone: one handle per graph, counted by itself
    alone = []
    for g in gs:
        with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
            alone.append(tuple(h.count()))
    assert alone == want
    ups = [chung_lu_graph(300 + 50 * j, 200 + 40 * j, 3000 + 500 * j, 2.2, 2.2, 0.3, seed=50 + j)
           for j in range(4)]
    up_want = [_want(g) for g in ups]
    # solo_wedges low enough that the largest graphs are counted alone
    with dbbc.Server(slots=4, max_batch=16, solo_wedges=2_000_000) as srv:
        ids = [srv.add_graph(g.n_u, g.n_v, g.u, g.v, g.sign) for g in gs]
        rng = np.random.default_rng(0)
        picks = rng.integers(0, len(gs), 600)
        tickets = []
        for n, i in enumerate(picks):
            tickets.append(("pool", int(i), srv.submit(ids[int(i)])))
            if n % 150 == 0:
                j = n // 150
                g = ups[j]
                tickets.append(("up", j, srv.submit_upload(g.n_u, g.n_v, g.u, g.v, g.sign)))
        sizes = []
        for kind, i, t in tickets:
            st, c, info = srv.wait(t)
            assert st == 0, (kind, i, info)
            assert tuple(c) == (want[i] if kind == "pool" else up_want[i]), (kind, i, info)
            assert info["t_submit_ns"] <= info["t_launch_ns"] <= info["t_done_ns"]
            sizes.append(info["batch_size"])
        s = srv.stats()
        _say("server stats", s, "max batch", max(sizes))
        assert s["completed"] == len(tickets) and s["failed"] == 0
        assert s["launches"] < len(tickets)     # requests shared launches
        assert max(sizes) > 1 and min(sizes) == 1
        assert s["uploads"] == len(ups)


def test_admission_by_footprint(dbbc):
    gs = [batch_graph(i) for i in range(3)]
    up = chung_lu_graph(2000, 1500, 40000, 2.2, 2.2, 0.3, seed=77)
    up_want = _want(up)
    def planned_bytes(g):
        with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
            h.count()
            return h.stats()["device_bytes"]
    pool = sum(planned_bytes(g) for g in gs)
    est = 64 * up.m + (1 << 20)  # the server's estimate for an upload
    # room for the pool, one upload's estimate and half an upload: each
    # upload after the first must evict the one before
    with dbbc.Server(hbm_budget=pool + est + planned_bytes(up) // 2) as srv:
        for g in gs:
            srv.add_graph(g.n_u, g.n_v, g.u, g.v, g.sign)
        res = []
        for _ in range(3):
            t = srv.submit_upload(up.n_u, up.n_v, up.u, up.v, up.sign)
            res.append(srv.wait(t))
        for st, c, info in res:
            assert st == 0 and tuple(c) == up_want, info
        s = srv.stats()
        _say("admission stats", s)
        assert s["evicted"] >= 1 and s["rejected"] == 0
    # a budget too small for any upload: rejected with DBBC_E_OOM
    with dbbc.Server(hbm_budget=1) as srv:
        t = srv.submit_upload(up.n_u, up.n_v, up.u, up.v, up.sign)
        st, c, info = srv.wait(t)
        assert st == dbbc.DBBC_E_OOM and c is None
        assert srv.stats()["rejected"] == 1
