"""GPU checks of the device text ingestion (dbbc_graph_create_text): the
paper's illustrative example written as records, texts with every format
variation the reader accepts, device-resident text, duplicates, malformed
lines and a full-size text; counts, per-vertex and per-edge outputs against
the oracle on the same edges, and the compact -> raw id maps against a
plain reading of the same text."""

import json
import os

import numpy as np
import pytest

from oracle import vp_counts
from synth import chung_lu_graph, config_graph, edge_text, messy_edge_text, raw_ids, uniform_graph

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


def _read_plain(text: bytes):
    """The records of a text as the format defines them, in plain Python:
    (raw u, raw v, sign) per non-skipped line, in line order."""
    recs = []
    for line in text.decode().split("\n"):
        f = line.replace(",", " ").replace("\t", " ").replace("\r", " ").split()
        if not f or f[0][0] in "#%":
            continue
        s = int(f[2])
        recs.append((int(f[0]), int(f[1]), 1 if s == 1 else -1))
    return recs


def test_paper_illustrative_example(dbbc):
    # Section IV-C: edges (2,5,0), (2,8,0), (7,5,0), (7,8,0): one balanced
    # butterfly; left ids {2, 7}, right ids {5, 8}
    text = b"2 5 0\n2 8 0\n7 5 0\n7 8 0\n"
    with dbbc.Graph.from_text(text) as h:
        c = h.count()
        assert (c.balanced, c.unbalanced, c.total) == (1, 0, 1)
        assert h.raw_ids(0).cpu().tolist() == [2, 7] and h.raw_ids(1).cpu().tolist() == [5, 8]
        assert h.info == {"lines": 4, "records": 4, "n_u": 2, "n_v": 2}


def test_fixture_graphs_as_text(dbbc):
    for name in ("fig_comparison.txt", "signed_k44.txt"):
        (fx,) = load(name)
        n_u, n_v, u, v, s = fx.arrays()
        r = vp_counts(n_u, n_v, u, v, s)
        with dbbc.Graph.from_text(edge_text(n_u, n_v, u, v, s)) as h:
            c = h.count()
        assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total), name


def test_messy_text_counts_and_maps(dbbc):
    for seed in range(6):
        g = chung_lu_graph(900, 700, 6000, 2.0, 1.8, 0.4, seed=seed)
        text, rec_lines = messy_edge_text(g.n_u, g.n_v, g.u, g.v, g.sign, seed=seed)
        recs = _read_plain(text)
        assert len(recs) == g.m
        _say("messy text", seed, len(text))
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True, per_edge=True)
        with dbbc.Graph.from_text(text) as h:
            c = h.count()
            assert (c.balanced, c.unbalanced, c.total) == (r.balanced, r.unbalanced, r.total)
            assert h.info["records"] == g.m and h.info["lines"] == text.count(b"\n") + (not text.endswith(b"\n"))
            ru, rv = h.raw_ids(0).cpu().numpy(), h.raw_ids(1).cpu().numpy()
            assert np.array_equal(ru, np.unique([a for a, _, _ in recs]))
            assert np.array_equal(rv, np.unique([b for _, b, _ in recs]))
            _, bu, bv, uu, uv = h.count_per_vertex()
            _, be, ue = h.count_per_edge()
        # compact id k of the text is the original vertex whose raw id is ru[k]
        inv_u = {int(x): i for i, x in enumerate(raw_ids(g.n_u, 0))}
        inv_v = {int(x): i for i, x in enumerate(raw_ids(g.n_v, 1))}
        ou = np.array([inv_u[int(x)] for x in ru])
        ov = np.array([inv_v[int(x)] for x in rv])
        assert np.array_equal(bu.cpu().numpy(), r.bal_u[ou]) and np.array_equal(uv.cpu().numpy(), r.unb_v[ov])
        assert np.array_equal(bv.cpu().numpy(), r.bal_v[ov]) and np.array_equal(uu.cpu().numpy(), r.unb_u[ou])
        # per-edge outputs follow the records
        assert np.array_equal(be.cpu().numpy(), r.bal_e) and np.array_equal(ue.cpu().numpy(), r.unb_e)


def test_device_text_and_duplicates(dbbc):
    import torch
    g = uniform_graph(300, 200, 4000, 0.3, seed=4)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    text = edge_text(g.n_u, g.n_v, g.u, g.v, g.sign)
    # the first 500 records repeated earlier with the opposite sign: the
    # later (original) record wins
    dup = edge_text(g.n_u, g.n_v, g.u[:500], g.v[:500], -g.sign[:500])
    t = torch.frombuffer(bytearray(dup + text), dtype=torch.uint8).to("cuda:0")
    with dbbc.Graph.from_text(t) as h:
        c = h.count()
        assert (c.balanced, c.unbalanced) == (r.balanced, r.unbalanced)
        assert h.stats()["dups_dropped"] == 500 and h.info["records"] == g.m + 500
    with pytest.raises(dbbc.DbbcError) as e:
        dbbc.Graph.from_text(dup + text, flags=dbbc.DBBC_DUP_REJECT)
    assert e.value.status == dbbc.DBBC_E_DUPLICATE


@pytest.mark.parametrize("bad,line", [
    (b"1 2 1\n3 4\n", 2),                      # missing sign
    (b"1 2 1\n\n3 4 2\n", 3),                  # sign out of range
    (b"# c\n1 x 1\n", 2),                      # not a number
    (b"1 2 -0\n", 1),                          # negative zero
    (b"1 2 1\n9223372036854775808 1 1\n", 2),  # id of 2^63
    (b"1 2 1\n1 2 1x\n", 2),                   # trailing junk in a field
])
def test_malformed_lines(dbbc, bad, line):
    with pytest.raises(dbbc.DbbcError) as e:
        dbbc.Graph.from_text(bad)
    assert e.value.status == dbbc.DBBC_E_PARSE and f"line {line}:" in str(e.value)


def test_texts_without_records(dbbc):
    for text in (b"", b"\n\n", b"% only\n# comments\n"):
        with pytest.raises(dbbc.DbbcError) as e:
            dbbc.Graph.from_text(text)
        assert e.value.status == dbbc.DBBC_E_INVALID_ARG


def test_powerlaw2m_text_full_size(dbbc):
    with open(os.path.join(GOLDEN, "oracle_cache.json")) as f:
        cache = json.load(f)["powerlaw2m"]
    g = config_graph("powerlaw2m")
    text = edge_text(g.n_u, g.n_v, g.u, g.v, g.sign)
    _say("powerlaw2m text", len(text))
    with dbbc.Graph.from_text(text) as h:
        c = h.count()
        st = h.stats()
    assert (c.balanced, c.unbalanced, c.total, c.wedges) == (cache["balanced"], cache["unbalanced"],
                                                             cache["total"], cache["wedges"])
    assert st["m"] == g.m
