"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every count is an exact integer, so the bar is equality.  Inputs are the
seeded synthetic graphs of synth/ and the paper's fixtures; the oracle runs
on the same arrays (or, for the 50M-edge workload, its counts come from
tests/golden/oracle_cache.json, written by a script that calls only the
oracle).
"""

import json
import os

import numpy as np
import pytest

from oracle import brute_counts, vp_counts
from synth import chung_lu_graph, config_graph, uniform_graph

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


def _gpu(dbbc, g, **opts):
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        return h.count(**opts)


def _want(g):
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    return (r.balanced, r.unbalanced, r.total, r.wedges)


def test_paper_fixtures(dbbc):
    for fname in ("k22_example.txt", "fig_comparison.txt", "fig_two.txt", "signed_k44.txt",
                  "drug_targets.txt"):
        for fx in load(fname):
            n_u, n_v, u, v, s = fx.arrays()
            _say("fixture", fname, fx.name)
            with dbbc.Graph(n_u, n_v, u, v, s) as h:
                got = h.count()
            b, ub, t = brute_counts(n_u, n_v, u, v, s)
            assert (got.balanced, got.unbalanced, got.total) == (b, ub, t), (fname, fx.name)
            exp = {e[0]: int(e[1]) for e in fx.expect if e[0] in ("balanced", "unbalanced")}
            for k, val in exp.items():
                assert getattr(got, k) == val


def test_random_small_graphs(dbbc):
    for seed in range(60):
        rng = np.random.default_rng(seed)
        if seed % 2:
            n_u, n_v = int(rng.integers(1, 40)), int(rng.integers(1, 40))
            g = uniform_graph(n_u, n_v, int(rng.integers(0, n_u * n_v + 1)), float(rng.random()),
                              seed=seed)
        else:
            g = chung_lu_graph(int(rng.integers(50, 800)), int(rng.integers(50, 800)),
                               int(rng.integers(100, 8000)), 2.0, 1.9, 0.4, seed=seed)
        _say("random graph", seed, g.n_u, g.n_v, g.m)
        want = _want(g)
        with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
            for opts in ({}, {"window_L": 256, "small_work": 2, "part_work": 4096},
                         {"window_L": 512, "small_work": 512, "reverse_L": 64},
                         {"window_L": 256, "long_len": 16}, {"long_len": 65536}):
                got = h.count(**opts)
                assert tuple(got) == want, (seed, opts)


@pytest.mark.parametrize("opts", [
    {}, {"window_L": 256}, {"window_L": 1024, "small_work": 2}, {"hub_T": 128, "window_L": 256},
    {"hub_T": 512, "window_L": 1024, "small_work": 64, "part_work": 4096},
    {"hub_T": 1024, "window_L": 32768}, {"window_L": 2048, "reverse_L": 64},
    {"window_L": 4096, "reverse_L": 4096, "small_work": 2},
    {"long_len": 16}, {"long_len": 65536, "window_L": 256}, {"long_len": 48, "small_work": 300},
])
def test_tiny_workload_option_sweep(dbbc, opts):
    g = config_graph("tiny")
    _say("tiny", opts)
    assert tuple(_gpu(dbbc, g, **opts)) == _want(g)


def test_dense_hub_block_paths(dbbc):
    # dense enough that most hub pairs get both dense and sparse wedges
    g = chung_lu_graph(1500, 1200, 150000, 2.4, 2.2, 0.35, seed=3)
    want = _want(g)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        for T in (0, 128, 256, 512, 1024):
            for L in (1024, 4096):
                _say("dense block", T, L)
                got = h.count(hub_T=T, window_L=L, part_work=4096)
                assert tuple(got) == want, (T, L)


def test_reverse_parts_and_windows(dbbc):
    # dense enough that reverse items exceed 127 segments (split into parts)
    g = chung_lu_graph(600, 500, 150000, 3.0, 3.0, 0.45, seed=9)
    want = _want(g)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        for opts in ({"window_L": 256, "reverse_L": 64}, {"window_L": 256, "reverse_L": 256},
                     {"window_L": 256, "reverse_L": 128, "hub_T": 128, "small_work": 2},
                     {"window_L": 512, "reverse_L": 192, "part_work": 4096}):
            _say("reverse parts", opts)
            assert tuple(h.count(**opts)) == want, opts


def test_powerlaw2m_full_size(dbbc):
    g = config_graph("powerlaw2m")
    want = _want(g)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        for opts in ({}, {"hub_T": 4096}, {"hub_T": 2048, "window_L": 8192}, {"hub_T": 0},
                     {"reverse_L": 1024}, {"window_L": 4096, "reverse_L": 4096},
                     {"long_len": 16}, {"long_len": 4096}, {"small_work": 8}):
            _say("powerlaw2m", opts)
            assert tuple(h.count(**opts)) == want, opts
        # repeated runs give identical integers (a race would show here)
        first = h.count()
        for _ in range(3):
            assert h.count() == first


def test_skewed50m_full_size(dbbc):
    with open(os.path.join(GOLDEN, "oracle_cache.json")) as f:
        cache = json.load(f)["skewed50m"]
    g = config_graph("skewed50m")
    assert (g.n_u, g.n_v, g.m) == (cache["n_u"], cache["n_v"], cache["m"])
    want = (cache["balanced"], cache["unbalanced"], cache["total"], cache["wedges"])
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        for opts in ({}, {"hub_T": 0}, {"hub_T": 4096}, {"reverse_L": 2048}):
            _say("skewed50m", opts)
            assert tuple(h.count(**opts)) == want, opts


def test_switching_and_relabel_on_gpu(dbbc):
    g = config_graph("powerlaw2m", scale=0.1)
    base = _gpu(dbbc, g)
    rng = np.random.default_rng(0)
    fu, fv = rng.random(g.n_u) < 0.5, rng.random(g.n_v) < 0.5
    s2 = (g.sign * np.where(fu[g.u] ^ fv[g.v], -1, 1)).astype(np.int8)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, s2) as h:
        assert h.count()[:3] == base[:3]
    with dbbc.Graph(g.n_v, g.n_u, g.v, g.u, g.sign) as h:  # sides swapped
        assert h.count()[:3] == base[:3]


def test_device_input_and_duplicates(dbbc):
    import torch
    g = config_graph("powerlaw2m", scale=0.05)
    want = _want(g)
    dev = torch.device("cuda:0")
    tu, tv, ts = (torch.from_numpy(a).to(dev) for a in (g.u, g.v, g.sign))
    with dbbc.Graph(g.n_u, g.n_v, tu, tv, ts) as h:
        assert tuple(h.count()) == want
        assert h.stats()["m"] == g.m
    # duplicates: the last record of a pair wins (the first 100 pairs are
    # listed first with the opposite sign, then with their real sign)
    u2 = np.concatenate([g.u[:100], g.u])
    v2 = np.concatenate([g.v[:100], g.v])
    s2 = np.concatenate([(-g.sign[:100]).astype(np.int8), g.sign])
    with dbbc.Graph(g.n_u, g.n_v, u2, v2, s2) as h:
        assert tuple(h.count()) == want
        assert h.stats()["dups_dropped"] == 100
    with pytest.raises(dbbc.DbbcError) as e:
        dbbc.Graph(g.n_u, g.n_v, u2, v2, s2, flags=dbbc.DBBC_DUP_REJECT)
    assert e.value.status == dbbc.DBBC_E_DUPLICATE


def test_edge_cases(dbbc):
    cases = [
        (1, 1, [], [], []),
        (3, 4, [0], [2], [-1]),
        (1, 50, [0] * 50, list(range(50)), [1] * 50),         # star: no butterfly
        (2, 2, [0, 0, 1, 1], [0, 1, 0, 1], [-1, -1, -1, 1]),  # one unbalanced
    ]
    for n_u, n_v, u, v, s in cases:
        u, v, s = (np.array(x, dt) for x, dt in ((u, np.int32), (v, np.int32), (s, np.int8)))
        _say("edge case", n_u, n_v, len(u))
        with dbbc.Graph(n_u, n_v, u, v, s) as h:
            got = h.count()
        r = vp_counts(n_u, n_v, u, v, s)
        assert tuple(got) == (r.balanced, r.unbalanced, r.total, r.wedges)
    # complete bipartite graph: closed form
    a, b = 300, 200
    uu, vv = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    with dbbc.Graph(a, b, uu.ravel(), vv.ravel(), np.ones(a * b, np.int8)) as h:
        full = (a * (a - 1) // 2) * (b * (b - 1) // 2)
        for opts in ({}, {"hub_T": 128, "window_L": 256}, {"window_L": 256, "part_work": 4096}):
            got = h.count(**opts)
            assert (got.balanced, got.unbalanced, got.total) == (full, 0, full), opts


def test_kernel_times(dbbc):
    g = config_graph("powerlaw2m", scale=0.2)
    with dbbc.Graph(g.n_u, g.n_v, g.u, g.v, g.sign) as h:
        h.count(flags=dbbc.DBBC_OPT_TIME_KERNELS, hub_T=1024)
        ks = h.kernel_times()
    names = [k["name"] for k in ks]
    assert {"direct", "reverse", "small", "hash", "reduce", "hub"} <= set(names)
    assert all(k["ms"] >= 0 for k in ks)
    assert sum(k["wedges"] for k in ks) > 0
    # one dense-block launch holds both sides: two contractions per tile
    hub = [k for k in ks if k["name"] == "hub"]
    assert len(hub) == 1 and hub[0]["macs"] > 0 and hub[0]["macs"] % (2 * 128 * 128) == 0
