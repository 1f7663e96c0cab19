"""GPU parity of the explicit-verification baseline (dbbc_count_explicit):
every pair of wedges checked on its signs gives exactly the oracle's counts
(the paper's fixtures, random graphs, the two stand-ins of the wedge-
separation study, degenerate graphs)."""

import numpy as np
import pytest

from oracle import vp_counts
from synth import chung_lu_graph, config_graph, uniform_graph

from golden_io import load

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


def _check(dbbc, n_u, n_v, u, v, s):
    r = vp_counts(n_u, n_v, u, v, s)
    with dbbc.Graph(n_u, n_v, u, v, s) as h:
        c = h.count_explicit()
        d = h.count()
    assert tuple(c) == (r.balanced, r.unbalanced, r.total, r.wedges) == tuple(d)


def test_fixtures(dbbc):
    for name in ("k22_example.txt", "fig_comparison.txt", "signed_k44.txt"):
        (fx,) = load(name)
        _check(dbbc, *fx.arrays())


def test_random_graphs(dbbc):
    for seed in range(12):
        rng = np.random.default_rng(2000 + seed)
        if seed % 2:
            g = uniform_graph(int(rng.integers(1, 60)), int(rng.integers(1, 60)),
                              int(rng.integers(0, 800)), float(rng.random()), seed=seed)
        else:
            g = chung_lu_graph(int(rng.integers(200, 3000)), int(rng.integers(200, 3000)),
                               int(rng.integers(500, 20000)), 2.0, 1.8, 0.4, seed=seed)
        _check(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign)


def test_study_stand_ins(dbbc):
    for name in ("se_like", "ho_like"):
        g = config_graph(name)
        print(name, flush=True)
        _check(dbbc, g.n_u, g.n_v, g.u, g.v, g.sign)


def test_degenerate(dbbc):
    for n_u, n_v, u, v, s in [(1, 1, [], [], []), (1, 30, [0] * 30, list(range(30)), [1] * 30),
                              (2, 2, [0, 0, 1, 1], [0, 1, 0, 1], [-1, 1, 1, 1])]:
        _check(dbbc, n_u, n_v, np.array(u, np.int32), np.array(v, np.int32), np.array(s, np.int8))
