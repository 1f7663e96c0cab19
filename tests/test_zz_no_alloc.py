"""dbbc_count_noalloc, through the C ABI: the count of dbbc_count with its
scratch in the library's per-GPU static array.  Two calls in a row, the
second on a smaller graph, each equal to dbbc_count's result and the
oracle's; then the refusals (no plan for the options, scratch too small)."""

import ctypes

import pytest

from oracle import vp_counts
from synth import chung_lu_graph

pytestmark = pytest.mark.gpu

E_INVALID_ARG, E_TOO_LARGE = -1, -7


@pytest.fixture(scope="module")
def dbbc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2609_21848_amd as mod
    mod.load()  # raises if the HIP library is missing
    return mod


def _noalloc(dbbc, h, opts):
    lib = dbbc.load()
    c = dbbc._Counts()
    o = dbbc.Options(**opts) if opts else None
    rc = lib.dbbc_count_noalloc(h.handle, ctypes.byref(o) if o is not None else None, ctypes.byref(c), None)
    return rc, (c.balanced, c.unbalanced, c.total, c.wedges)


OPTS = ({}, {"hub_T": 256, "window_L": 1024},
        {"window_L": 256, "reverse_L": 64, "small_work": 2, "part_work": 4096})


@pytest.mark.parametrize("opts", OPTS)
def test_noalloc_equals_count_twice_smaller_second(dbbc, opts):
    big = chung_lu_graph(6000, 5000, 120000, 2.1, 1.9, 0.4, seed=31)
    small = chung_lu_graph(900, 700, 9000, 2.2, 2.0, 0.3, seed=32)
    print("noalloc", opts, flush=True)
    with dbbc.Graph(big.n_u, big.n_v, big.u, big.v, big.sign) as hb, \
            dbbc.Graph(small.n_u, small.n_v, small.u, small.v, small.sign) as hs:
        want_b, want_s = tuple(hb.count(**opts)), tuple(hs.count(**opts))  # plans both
        rc, got_b = _noalloc(dbbc, hb, opts)
        assert rc == 0, dbbc.load().dbbc_last_error()
        rc, got_s = _noalloc(dbbc, hs, opts)
        assert rc == 0, dbbc.load().dbbc_last_error()
        assert got_b == want_b and got_s == want_s
        # again, in the other order: the array keeps the last call's contents
        assert _noalloc(dbbc, hb, opts) == (0, want_b)
    for g, got in ((big, got_b), (small, got_s)):
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
        assert got == (r.balanced, r.unbalanced, r.total, r.wedges)


def test_noalloc_refusals(dbbc):
    g = chung_lu_graph(6000, 5000, 120000, 2.1, 1.9, 0.4, seed=31)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        # not planned for these options: refused, nothing runs
        rc, _ = _noalloc(dbbc, h, {"window_L": 512})
        assert rc == E_INVALID_ARG
        assert "plan" in dbbc.load().dbbc_last_error().decode()
        # two sides' 2048 x 2048 hub-pair planes alone fill the 64 MiB array
        h.count(hub_T=2048)
        rc, _ = _noalloc(dbbc, h, {"hub_T": 2048})
        assert rc == E_TOO_LARGE
        assert "scratch" in dbbc.load().dbbc_last_error().decode()
        # the graph is untouched: a plain count still gives the oracle's result
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
        assert tuple(h.count(hub_T=2048)) == (r.balanced, r.unbalanced, r.total, r.wedges)
