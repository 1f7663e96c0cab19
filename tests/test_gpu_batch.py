"""GPU parity of batched counts: many graphs through one launch sequence
(optionally captured into a HIP graph and replayed) must give, graph by
graph, exactly the oracle's counts and the counts of each graph alone."""

import numpy as np
import pytest

from oracle import vp_counts
from synth import batch_graph, chung_lu_graph, uniform_graph

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


def _mixed_graphs():
    """Uneven sizes, empty and one-edge graphs, and graphs dense enough for
    the dense hub block and for reverse parts."""
    gs = [uniform_graph(3, 4, 0, 0.5, seed=1), uniform_graph(1, 1, 1, 0.5, seed=2),
          uniform_graph(2, 2, 4, 1.0, seed=3)]
    for seed in range(12):
        rng = np.random.default_rng(100 + seed)
        gs.append(chung_lu_graph(int(rng.integers(20, 2500)), int(rng.integers(20, 2500)),
                                 int(rng.integers(50, 20000)), 2.0, 1.9, float(rng.random()),
                                 seed=seed))
    gs.append(chung_lu_graph(1500, 1200, 150000, 2.4, 2.2, 0.35, seed=3))
    gs.append(chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9))
    for i in range(6):
        gs.append(batch_graph(i * 511))
    return gs


@pytest.mark.parametrize("opts", [{}, {"hub_T": 128, "window_L": 256, "small_work": 64},
                                  {"window_L": 512, "reverse_L": 128, "part_work": 4096}])
def test_batch_matches_oracle_and_lone_counts(dbbc, opts):
    gs = _mixed_graphs()
    want = [_want(g) for g in gs]
    hs = [dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) for g in gs]
    try:
        _say("batch", len(hs), opts)
        with dbbc.Batch(hs, **opts) as b:
            got = b.count()
        assert [tuple(c) for c in got] == want
        # each graph alone (same plan) gives the same integers
        for h, w in zip(hs, want):
            assert tuple(h.count(**opts)) == w
        # the one-shot form
        got = dbbc.dbbc_count_batch(hs, dbbc.Options(**opts))
        assert [tuple(c) for c in got] == want
    finally:
        for h in hs:
            h.close()


def test_captured_batch_replays(dbbc):
    import torch
    gs = [batch_graph(i) for i in range(0, 4096, 97)]
    want = [_want(g) for g in gs]
    hs = [dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) for g in gs]
    stream = torch.cuda.Stream()
    try:
        with dbbc.Batch(hs, capture=True, stream=stream) as b:
            for rep in range(5):
                _say("replay", rep)
                with torch.cuda.stream(stream):
                    # the program's own eager device work between replays
                    x = torch.randn(1 << 20, device="cuda", generator=None)
                    y = (x * 2).sum()
                got = b.count(stream=stream)
                assert [tuple(c) for c in got] == want, rep
                torch.cuda.synchronize()
                assert torch.isfinite(y)
            # asynchronous form
            b.launch(stream=stream)
            stream.synchronize()
            assert [tuple(c) for c in b.read()] == want
    finally:
        for h in hs:
            h.close()


def test_batch_rejects_duplicates_and_replans(dbbc):
    gs = [batch_graph(1), batch_graph(2)]
    hs = [dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) for g in gs]
    try:
        with pytest.raises(dbbc.DbbcError):
            dbbc.Batch([hs[0], hs[1], hs[0]])
        b = dbbc.Batch(hs)
        want = [tuple(c) for c in b.count()]
        hs[1].count(window_L=256)  # a new plan for graph 1
        with pytest.raises(dbbc.DbbcError):
            b.count()
        b.close()
        with dbbc.Batch(hs, window_L=256) as b2:
            assert [tuple(c) for c in b2.count()] == want
        with dbbc.Batch([]) as b3:
            assert b3.count() == []
    finally:
        for h in hs:
            h.close()


def test_async_lone_counts(dbbc):
    import torch
    gs = [batch_graph(i) for i in (5, 6, 7)]
    want = [_want(g) for g in gs]
    hs = [dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) for g in gs]
    streams = [torch.cuda.Stream() for _ in hs]
    try:
        for h, s in zip(hs, streams):
            h.count_async(stream=s)
        with pytest.raises(dbbc.DbbcError):
            hs[0].count()  # a count is in flight on this handle
        for s in streams:
            s.synchronize()
        assert [tuple(h.read()) for h in hs] == want
        with pytest.raises(dbbc.DbbcError):
            hs[0].read()  # nothing in flight any more
    finally:
        for h in hs:
            h.close()


def test_autotune_keeps_counts(dbbc):
    gs = [batch_graph(i) for i in range(0, 4096, 257)]
    want = [_want(g) for g in gs]
    hs = [dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) for g in gs]
    try:
        best, ms = dbbc.dbbc_autotune(hs, reps=2)
        _say("autotune", best, ms)
        assert ms > 0
        with dbbc.Batch(hs, capture=True, **best) as b:
            assert [tuple(c) for c in b.count()] == want
        assert [tuple(h.count(**best)) for h in hs] == want
    finally:
        for h in hs:
            h.close()
