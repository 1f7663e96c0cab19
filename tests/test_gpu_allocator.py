"""The device allocator hook (dbbc_allocator, through the C ABI): every device
allocation a handle or a batch makes goes through the caller's functions,
every block comes back to them, and the counts equal the oracle's and those
of the default allocator (hipMalloc)."""

import numpy as np
import pytest

from oracle import vp_counts
from synth import chung_lu_graph

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


class Counting:
    """An allocator over PyTorch's caching allocator that records every block."""

    def __init__(self, dbbc):
        import torch
        self.live, self.errors = {}, []
        self.n_alloc = self.n_free = 0

        def alloc(nbytes, stream, ctx):
            p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                   int(stream or 0))
            self.live[p] = int(nbytes)
            self.n_alloc += 1
            return p

        def free(ptr, stream, ctx):
            if ptr not in self.live:
                self.errors.append(f"free of unknown block {ptr:#x}")
                return
            del self.live[ptr]
            self.n_free += 1
            torch.cuda.caching_allocator_delete(int(ptr))

        self.struct = dbbc.Allocator(dbbc._ALLOC_FN(alloc), dbbc._FREE_FN(free), None)


def _want(r):
    return (r.balanced, r.unbalanced, r.total, r.wedges)


def test_counting_allocator_sees_every_block_back(dbbc):
    from synth import edge_text
    g = chung_lu_graph(3000, 2000, 40000, 2.1, 1.9, 0.4, seed=11)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True, per_edge=True)
    ca = Counting(dbbc)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign, allocator=ca.struct) as h:
        assert ca.n_alloc > 0 and ca.n_free > 0, "the build's arrays should come and go"
        held = len(ca.live)
        assert tuple(h.count()) == _want(r)
        assert len(ca.live) > held, "the plan should come from the allocator"
        assert tuple(h.count(hub_T=256, window_L=1024)) == _want(r)  # re-planned
        c, bu, bv, uu, uv = h.count_per_vertex()
        assert tuple(c) == _want(r)
        for t, want in ((bu, r.bal_u), (bv, r.bal_v), (uu, r.unb_u), (uv, r.unb_v)):
            assert np.array_equal(t.cpu().numpy(), want)
        c, be, ue = h.count_per_edge()
        assert np.array_equal(be.cpu().numpy(), r.bal_e) and np.array_equal(ue.cpu().numpy(), r.unb_e)
        assert tuple(h.count_explicit()) == _want(r)
        with dbbc.Batch([h], capture=True) as b:
            assert tuple(b.count()[0]) == _want(r)
        with dbbc.Graph.from_text(edge_text(g.n_u, g.n_v, g.u, g.v, g.sign),
                                  allocator=ca.struct) as ht:
            assert tuple(ht.count()) == _want(r)
    assert not ca.errors, ca.errors
    assert ca.live == {} and ca.n_free == ca.n_alloc


def test_default_allocator_same_counts(dbbc):
    g = chung_lu_graph(3000, 2000, 40000, 2.1, 1.9, 0.4, seed=12)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    for alloc in (None, "torch"):
        with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign, allocator=alloc) as h:
            assert tuple(h.count()) == _want(r)
            assert tuple(h.count(hub_T=256, window_L=1024)) == _want(r)
