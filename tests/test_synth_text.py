"""The text writers of synth/ (CPU): every record of a written text reads
back, in order, as the same edge under the id map, in both writers."""

import numpy as np

from synth import chung_lu_graph, edge_text, messy_edge_text, raw_ids


def _records(text: bytes):
    out = []
    for line in text.decode().split("\n"):
        f = line.replace(",", " ").replace("\t", " ").replace("\r", " ").split()
        if f and f[0][0] not in "#%":
            out.append((int(f[0]), int(f[1]), 1 if int(f[2]) == 1 else -1))
    return out


def test_writers_round_trip():
    g = chung_lu_graph(400, 300, 3000, 2.0, 1.8, 0.4, seed=3)
    want = list(zip(raw_ids(g.n_u, 0)[g.u].tolist(), raw_ids(g.n_v, 1)[g.v].tolist(), g.sign.tolist()))
    assert _records(edge_text(g.n_u, g.n_v, g.u, g.v, g.sign)) == want
    for seed in range(3):
        text, rec_lines = messy_edge_text(g.n_u, g.n_v, g.u, g.v, g.sign, seed=seed)
        assert _records(text) == want
        assert len(rec_lines) == g.m and rec_lines == sorted(rec_lines)


def test_raw_ids_are_distinct():
    for side in (0, 1):
        r = raw_ids(100000, side)
        assert np.unique(r).size == r.size and r.min() >= 0 and r.max() < (1 << 40)


def test_sign_probability_keeps_topology():
    """The sign-ratio study varies only the signs of one topology."""
    import numpy as np
    from synth import config_graph
    a = config_graph("powerlaw2m", scale=0.05, q=0.1)
    b = config_graph("powerlaw2m", scale=0.05, q=0.9)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v)
    assert (a.sign < 0).mean() < 0.15 and (b.sign < 0).mean() > 0.85
