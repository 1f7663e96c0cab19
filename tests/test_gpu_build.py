"""GPU checks of the device graph build (dedup, degrees, priority relabel,
CSR pair, reverse positions, cut, W_VP): record validation through the C
ABI, the handle's statistics against plain computations and the oracle, and
counts on graphs that stress the relabel (isolated vertices, degree ties,
one-vertex sides, device input with duplicates)."""

import numpy as np
import pytest

from oracle import vp_counts
from synth import chung_lu_graph, uniform_graph

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


def _err(dbbc, *args, **kw):
    with pytest.raises(dbbc.DbbcError) as e:
        dbbc.Graph(*args, **kw)
    return e.value


def test_record_validation(dbbc):
    import torch
    i32, i8 = np.int32, np.int8
    e = _err(dbbc, 2, 2, np.array([0, 2], i32), np.array([0, 1], i32), np.array([1, 1], i8))
    assert e.status == dbbc.DBBC_E_ID_RANGE and "edge 1" in str(e)
    e = _err(dbbc, 2, 2, np.array([0, 1], i32), np.array([0, -1], i32), np.array([1, 1], i8))
    assert e.status == dbbc.DBBC_E_ID_RANGE
    e = _err(dbbc, 2, 2, np.array([0, 1], i32), np.array([0, 1], i32), np.array([1, 0], i8))
    assert e.status == dbbc.DBBC_E_SIGN and "edge 1" in str(e) and "sign 0" in str(e)
    # the first bad record decides, ids before signs
    e = _err(dbbc, 3, 3, np.array([0, 0, 5, 0], i32), np.array([0, 1, 0, 2], i32),
             np.array([1, 3, 1, 1], i8))
    assert e.status == dbbc.DBBC_E_SIGN and "edge 1" in str(e)
    e = _err(dbbc, 3, 3, np.array([0, 7, 0], i32), np.array([0, 1, 0], i32), np.array([1, 2, 1], i8))
    assert e.status == dbbc.DBBC_E_ID_RANGE and "edge 1" in str(e)
    e = _err(dbbc, 2, 2, np.array([0, 1, 0], i32), np.array([0, 1, 0], i32), np.array([1, 1, -1], i8),
             flags=dbbc.DBBC_DUP_REJECT)
    assert e.status == dbbc.DBBC_E_DUPLICATE and "duplicate" in str(e)
    dev = torch.device("cuda:0")
    e = _err(dbbc, 2, 2, torch.tensor([0, 1], dtype=torch.int32, device=dev),
             torch.tensor([0, 3], dtype=torch.int32, device=dev),
             torch.tensor([1, 1], dtype=torch.int8, device=dev))
    assert e.status == dbbc.DBBC_E_ID_RANGE


def _stats_check(dbbc, n_u, n_v, u, v, s):
    r = vp_counts(n_u, n_v, u, v, s)
    with dbbc.Graph(n_u, n_v, u, v, s) as h:
        st = h.stats()
        c = h.count()
    assert tuple(c) == (r.balanced, r.unbalanced, r.total, r.wedges)
    assert st["wedges_vp"] == r.wedges and st["m"] == len(u) and st["dups_dropped"] == 0
    du = np.bincount(u, minlength=n_u)
    dv = np.bincount(v, minlength=n_v)
    assert st["max_deg_u"] == int(du.max(initial=0)) and st["max_deg_v"] == int(dv.max(initial=0))


def test_stats_and_counts_on_relabel_edge_cases(dbbc):
    rng = np.random.default_rng(3)
    # isolated vertices on both sides, many degree ties
    g = uniform_graph(5000, 4000, 6000, 0.5, seed=3)
    _stats_check(dbbc, 20000, 30000, g.u, g.v, g.sign)
    # one vertex on a side
    v = np.arange(40, dtype=np.int32)
    _stats_check(dbbc, 1, 40, np.zeros(40, np.int32), v, rng.choice([-1, 1], 40).astype(np.int8))
    _stats_check(dbbc, 40, 1, v, np.zeros(40, np.int32), rng.choice([-1, 1], 40).astype(np.int8))
    # regular graph: every degree equal, order by id only
    a = np.repeat(np.arange(300, dtype=np.int32), 6)
    b = ((a * 7 + np.tile(np.arange(6), 300) * 53) % 300).astype(np.int32)
    _stats_check(dbbc, 300, 300, a, b, rng.choice([-1, 1], a.size).astype(np.int8))
    # skewed graphs of several sizes
    for seed in range(4):
        g = chung_lu_graph(3000 + 1000 * seed, 2000, 40000, 2.0, 1.8, 0.4, seed=seed)
        _stats_check(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign)


def test_device_input_shuffled_with_duplicates(dbbc):
    import torch
    g = chung_lu_graph(4000, 3000, 50000, 2.0, 1.9, 0.4, seed=8)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_edge=True)
    rng = np.random.default_rng(8)
    dup = rng.choice(g.m, 5000, replace=False)
    # each duplicated pair appears first with the opposite sign at a random
    # earlier place; the original record (kept, last) keeps its position
    # after every copy
    order = rng.permutation(g.m)
    u = np.concatenate([g.u[dup], g.u[order]]).astype(np.int32)
    v = np.concatenate([g.v[dup], g.v[order]]).astype(np.int32)
    s = np.concatenate([-g.sign[dup], g.sign[order]]).astype(np.int8)
    dev = torch.device("cuda:0")
    tu, tv, ts = (torch.from_numpy(x).to(dev) for x in (u, v, s))
    with dbbc.Graph(g.n_u, g.n_v, tu, tv, ts) as h:
        c, be, ue = h.count_per_edge()
        assert h.stats()["dups_dropped"] == 5000 and h.stats()["m"] == g.m
    assert (c.balanced, c.unbalanced) == (r.balanced, r.unbalanced)
    be, ue = be.cpu().numpy(), ue.cpu().numpy()
    assert (be[:5000] == 0).all() and (ue[:5000] == 0).all()
    assert np.array_equal(be[5000:], r.bal_e[order]) and np.array_equal(ue[5000:], r.unb_e[order])
