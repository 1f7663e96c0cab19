"""Pins for the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the fixtures carry the paper's
printed values (or values derived by hand, said so in the fixture), the
closed forms are counted by hand, and the three oracle tiers are independent
formulations (Definitions 1-2 brute force, the Lemma 1 pair form, and
Algorithm 1's vertex-priority enumeration).
"""

from math import comb

import numpy as np
import pytest

from oracle import (brute_counts, brute_per_edge, brute_per_vertex, edge_counts_at, pair_counts,
                    pair_per_vertex, vp_counts)
from synth import chung_lu_graph, config_graph, uniform_graph

from golden_io import load


def _all_tiers(n_u, n_v, u, v, s):
    res = {
        "brute": brute_counts(n_u, n_v, u, v, s),
        "pairs_u": pair_counts(n_u, n_v, u, v, s, "u", "dense"),
        "pairs_v": pair_counts(n_u, n_v, u, v, s, "v", "sparse"),
    }
    r = vp_counts(n_u, n_v, u, v, s, threads=2)
    res["vp"] = (r.balanced, r.unbalanced, r.total)
    return res


# --- fixtures from the paper ---------------------------------------------------

def test_k22_illustrative_example():
    (fx,) = load("k22_example.txt")
    n_u, n_v, u, v, s = fx.arrays()
    ids = np.array([int(k) for k in fx.left] + [int(k) for k in fx.right], np.int64)
    exp = {e[0]: e[1:] for e in fx.expect if e[0] != "pivot_balanced"}
    want = tuple(int(exp[k][0]) for k in ("balanced", "unbalanced", "total"))
    for tier, got in _all_tiers(n_u, n_v, u, v, s).items():
        assert got == want, tier
    r = vp_counts(n_u, n_v, u, v, s, ids=ids, per_pivot=True, threads=1)
    for e in fx.expect:
        if e[0] == "pivot_balanced":
            assert r.per_pivot_bal[fx.vertex(e[1])] == int(e[2]), e
    # Every edge is expanded exactly once, from its higher-priority endpoint
    # (complexity analysis); the three surviving wedges are 8-2-5, 8-7-5, 7-5-2.
    assert r.expansions == 4
    assert r.wedges == 3


def test_fig_comparison_vertex_and_edge_counts():
    (fx,) = load("fig_comparison.txt")
    n_u, n_v, u, v, s = fx.arrays()
    bu, bv, uu, uv = brute_per_vertex(n_u, n_v, u, v, s)
    pu, pv, _, _ = pair_per_vertex(n_u, n_v, u, v, s)
    r = vp_counts(n_u, n_v, u, v, s, per_vertex=True, per_edge=True, threads=2)
    be, ue = brute_per_edge(n_u, n_v, u, v, s)
    edge_index = {(a, b): i for i, (a, b, _) in enumerate(fx.edges)}
    for e in fx.expect:
        if e[0] == "vertex_balanced":
            x = fx.vertex(e[1])
            assert bu[x] == pu[x] == r.bal_u[x] == int(e[2]), e
        elif e[0] == "edge_balanced":
            i = edge_index[(fx.left[e[1]], fx.right[e[2]])]
            assert be[i] == r.bal_e[i] == int(e[3]), e
    # edges the figure does not list lie in no balanced butterfly
    listed = {edge_index[(fx.left[e[1]], fx.right[e[2]])] for e in fx.expect
              if e[0] == "edge_balanced"}
    assert all(r.bal_e[i] == be[i] == 0 for i in range(len(fx.edges)) if i not in listed)
    assert list(r.unb_e) == list(ue) == [0] * len(fx.edges)
    # Right-side values follow from the same figure (each of 1, 2, 5, 6 lies
    # in three balanced butterflies, 3 and 4 in one).
    assert list(bv) == list(pv) == list(r.bal_v) == [3, 3, 1, 1, 3, 3]
    assert r.balanced == 7 and r.unbalanced == 0


@pytest.mark.parametrize("fname", ["fig_two.txt", "drug_targets.txt"])
def test_single_butterfly_classes(fname):
    graphs = load(fname)
    assert len(graphs) >= 4
    for fx in graphs:
        n_u, n_v, u, v, s = fx.arrays()
        want = (1, 0, 1) if fx.label == "balanced" else (0, 1, 1)
        for tier, got in _all_tiers(n_u, n_v, u, v, s).items():
            assert got == want, (fx.name, tier)


def test_signed_k44():
    (fx,) = load("signed_k44.txt")
    n_u, n_v, u, v, s = fx.arrays()
    exp = {e[0]: int(e[1]) for e in fx.expect}
    for tier, got in _all_tiers(n_u, n_v, u, v, s).items():
        assert got == (exp["balanced"], exp["unbalanced"], exp["total"]), tier


def test_all_sixteen_sign_patterns_of_one_butterfly():
    # Definition 2 by exhaustion: 8 of the 16 sign patterns have an even
    # number of negative edges.
    u = np.array([0, 0, 1, 1], np.int32)
    v = np.array([0, 1, 0, 1], np.int32)
    n_bal = 0
    for mask in range(16):
        s = np.array([-1 if (mask >> i) & 1 else 1 for i in range(4)], np.int8)
        k = bin(mask).count("1")
        r = vp_counts(2, 2, u, v, s, threads=1)
        assert (r.balanced, r.unbalanced) == ((1, 0) if k % 2 == 0 else (0, 1))
        assert brute_counts(2, 2, u, v, s)[:2] == (r.balanced, r.unbalanced)
        n_bal += r.balanced
    assert n_bal == 8


# --- closed forms ---------------------------------------------------------------

def _complete(a, b):
    uu, vv = np.meshgrid(np.arange(a), np.arange(b), indexing="ij")
    return uu.ravel().astype(np.int32), vv.ravel().astype(np.int32)


@pytest.mark.parametrize("a,b", [(2, 2), (3, 5), (7, 4), (12, 9), (30, 2)])
def test_complete_bipartite_closed_forms(a, b):
    u, v = _complete(a, b)
    full = comb(a, 2) * comb(b, 2)
    for sgn in (1, -1):
        s = np.full(u.shape, sgn, np.int8)
        r = vp_counts(a, b, u, v, s, threads=2)
        assert (r.balanced, r.unbalanced, r.total) == (full, 0, full)
    # exactly one negative edge: it lies in (a-1)(b-1) butterflies, each with
    # one negative edge
    s = np.ones(u.shape, np.int8)
    s[0] = -1
    r = vp_counts(a, b, u, v, s, threads=2)
    assert r.unbalanced == (a - 1) * (b - 1)
    assert r.balanced == full - (a - 1) * (b - 1)
    # s(u, v) = x_u * y_v: every 4-cycle's sign product is a square, so +1
    rng = np.random.default_rng(a * 100 + b)
    x = rng.choice([-1, 1], a)
    y = rng.choice([-1, 1], b)
    s = (x[u] * y[v]).astype(np.int8)
    r = vp_counts(a, b, u, v, s, threads=2)
    assert (r.balanced, r.unbalanced) == (full, 0)
    # each edge is expanded once from its higher-priority end
    assert r.expansions == a * b


@pytest.mark.parametrize("a,b", [(2, 2), (3, 5), (7, 4), (9, 6)])
def test_complete_bipartite_per_edge_closed_forms(a, b):
    u, v = _complete(a, b)
    k = (a - 1) * (b - 1)  # butterflies through one edge of K(a,b)
    r = vp_counts(a, b, u, v, np.ones(u.shape, np.int8), per_edge=True, threads=2)
    assert (r.bal_e == k).all() and (r.unb_e == 0).all()
    # one negative edge e0 = (0, 0): every butterfly through e0 is unbalanced;
    # an edge (0, y) meets e0 in a-1 butterflies (any second U vertex, V pair
    # fixed), an edge (x, 0) in b-1, an edge disjoint from e0 in exactly one
    s = np.ones(u.shape, np.int8)
    s[0] = -1
    r = vp_counts(a, b, u, v, s, per_edge=True, threads=2)
    for i in range(u.shape[0]):
        x, y = int(u[i]), int(v[i])
        with_e0 = k if (x, y) == (0, 0) else (a - 1 if x == 0 else b - 1 if y == 0 else 1)
        assert (r.unb_e[i], r.bal_e[i]) == (with_e0, k - with_e0), (i, x, y)


# --- agreement of the three tiers --------------------------------------------------

def test_tiers_agree_on_random_tiny_graphs():
    for seed in range(240):
        rng = np.random.default_rng(seed)
        n_u, n_v = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        m = int(rng.integers(0, n_u * n_v + 1))
        g = uniform_graph(n_u, n_v, m, float(rng.random()), seed=seed)
        got = _all_tiers(g.n_u, g.n_v, g.u, g.v, g.sign)
        assert len(set(got.values())) == 1, (seed, got)
        if seed % 4 == 0:
            bvx = brute_per_vertex(g.n_u, g.n_v, g.u, g.v, g.sign)
            r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True, per_edge=True,
                          threads=2)
            pvx = pair_per_vertex(g.n_u, g.n_v, g.u, g.v, g.sign)
            for a, b, c in zip(bvx, pvx, (r.bal_u, r.bal_v, r.unb_u, r.unb_v)):
                assert list(a) == list(b) == list(c), seed
            be, ue = brute_per_edge(g.n_u, g.n_v, g.u, g.v, g.sign)
            assert list(r.bal_e) == be and list(r.unb_e) == ue, seed
            lb, lu = edge_counts_at(g.n_u, g.n_v, g.u, g.v, g.sign, range(g.m))
            assert lb == be and lu == ue, seed


def test_tiers_agree_on_skewed_small_graphs():
    for seed in range(20):
        g = chung_lu_graph(30, 25, 200, 2.0, 1.9, 0.4, seed=seed)
        got = _all_tiers(g.n_u, g.n_v, g.u, g.v, g.sign)
        assert len(set(got.values())) == 1, (seed, got)


def test_tiny_uniform_workload_pair_form_equals_vp():
    g = config_graph("tiny")
    dense_u = pair_counts(g.n_u, g.n_v, g.u, g.v, g.sign, "u", "dense")
    dense_v = pair_counts(g.n_u, g.n_v, g.u, g.v, g.sign, "v", "dense")
    sparse = pair_counts(g.n_u, g.n_v, g.u, g.v, g.sign, "u", "sparse")
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    assert dense_u == dense_v == sparse == (r.balanced, r.unbalanced, r.total)
    assert r.expansions == g.m


# --- invariants --------------------------------------------------------------------

def _graph(seed, n_u=300, n_v=200, m=3000):
    return chung_lu_graph(n_u, n_v, m, 2.1, 2.0, 0.35, seed=seed)


def _vp(n_u, n_v, u, v, s, **kw):
    r = vp_counts(n_u, n_v, u, v, s, threads=4, **kw)
    return r


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_invariants(seed):
    g = _graph(seed)
    base = _vp(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True, per_edge=True)
    assert base.balanced + base.unbalanced == base.total
    assert base.expansions == g.m
    # unsigned total = the count with every sign positive
    plus = _vp(g.n_u, g.n_v, g.u, g.v, np.ones(g.m, np.int8))
    assert (plus.balanced, plus.unbalanced) == (base.total, 0)
    # per-vertex sums: every butterfly has two vertices on each side
    for arr, tot in ((base.bal_u, base.balanced), (base.bal_v, base.balanced),
                     (base.unb_u, base.unbalanced), (base.unb_v, base.unbalanced)):
        assert int(arr.sum()) == 2 * tot
    # per-edge sums: four edges per butterfly, and two of them at each of its
    # vertices
    assert int(base.bal_e.sum()) == 4 * base.balanced
    assert int(base.unb_e.sum()) == 4 * base.unbalanced
    some = np.random.default_rng(seed + 17).choice(g.m, 40, replace=False)
    lb, lu = edge_counts_at(g.n_u, g.n_v, g.u, g.v, g.sign, some)
    assert lb == list(base.bal_e[some]) and lu == list(base.unb_e[some])
    for per_e, pu_, pv_ in ((base.bal_e, base.bal_u, base.bal_v),
                            (base.unb_e, base.unb_u, base.unb_v)):
        assert np.array_equal(np.bincount(g.u, per_e, g.n_u).astype(np.int64), 2 * pu_)
        assert np.array_equal(np.bincount(g.v, per_e, g.n_v).astype(np.int64), 2 * pv_)
    rng = np.random.default_rng(seed)
    # switching: negate every edge at a random set of vertices
    flip_u = rng.random(g.n_u) < 0.5
    flip_v = rng.random(g.n_v) < 0.5
    s2 = g.sign * np.where(flip_u[g.u] ^ flip_v[g.v], -1, 1).astype(np.int8)
    sw = _vp(g.n_u, g.n_v, g.u, g.v, s2, per_vertex=True, per_edge=True)
    assert (sw.balanced, sw.unbalanced) == (base.balanced, base.unbalanced)
    assert np.array_equal(sw.bal_u, base.bal_u) and np.array_equal(sw.unb_v, base.unb_v)
    assert np.array_equal(sw.bal_e, base.bal_e) and np.array_equal(sw.unb_e, base.unb_e)
    # any strict total order (Theorem 1): random tie-break ids and random
    # degree-free orders give the same totals
    ids = rng.permutation(g.n_u + g.n_v).astype(np.int64)
    r = _vp(g.n_u, g.n_v, g.u, g.v, g.sign, ids=ids)
    assert (r.balanced, r.unbalanced) == (base.balanced, base.unbalanced)
    # relabelling the vertices of each side and swapping the sides
    pu = rng.permutation(g.n_u).astype(np.int32)
    pv = rng.permutation(g.n_v).astype(np.int32)
    r = _vp(g.n_u, g.n_v, pu[g.u], pv[g.v], g.sign)
    assert (r.balanced, r.unbalanced) == (base.balanced, base.unbalanced)
    r = _vp(g.n_v, g.n_u, g.v, g.u, g.sign)
    assert (r.balanced, r.unbalanced) == (base.balanced, base.unbalanced)
    # edge order does not matter
    perm = rng.permutation(g.m)
    r = _vp(g.n_u, g.n_v, g.u[perm], g.v[perm], g.sign[perm], per_edge=True)
    assert (r.balanced, r.unbalanced, r.wedges) == (base.balanced, base.unbalanced, base.wedges)
    assert np.array_equal(r.bal_e, base.bal_e[perm]) and np.array_equal(r.unb_e, base.unb_e[perm])


def test_disjoint_union_is_additive():
    a, b = _graph(5), _graph(6, 150, 400, 2500)
    ra = _vp(a.n_u, a.n_v, a.u, a.v, a.sign)
    rb = _vp(b.n_u, b.n_v, b.u, b.v, b.sign)
    u = np.concatenate([a.u, b.u + a.n_u]).astype(np.int32)
    v = np.concatenate([a.v, b.v + a.n_v]).astype(np.int32)
    s = np.concatenate([a.sign, b.sign])
    r = _vp(a.n_u + b.n_u, a.n_v + b.n_v, u, v, s)
    assert (r.balanced, r.unbalanced, r.wedges) == (
        ra.balanced + rb.balanced, ra.unbalanced + rb.unbalanced, ra.wedges + rb.wedges)


def _wedges_closed_form(n_u, n_v, u, v):
    """Sum over edges (x, y), x of higher priority, of the number of
    neighbours of y ranked below x: d(y) - 1 - (position of x in y's
    neighbour list sorted from highest to lowest priority)."""
    n = n_u + n_v
    a = u.astype(np.int64)
    b = n_u + v.astype(np.int64)
    deg = np.bincount(np.concatenate([a, b]), minlength=n)
    gid = np.arange(n)
    order = np.lexsort((-gid, -deg))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    total = 0
    for hi_, lo_ in ((a, b), (b, a)):
        # edges seen from lo_'s neighbour list; expansions come from hi_ when
        # rank[hi_] < rank[lo_]
        o = np.lexsort((rank[hi_], lo_))
        lo_s, hi_s = lo_[o], hi_[o]
        start = np.searchsorted(lo_s, lo_s, side="left")
        pos = np.arange(lo_s.shape[0]) - start
        cnt = deg[lo_s] - 1 - pos
        total += int(cnt[rank[hi_s] < rank[lo_s]].sum())
    return total


@pytest.mark.parametrize("seed", [0, 3])
def test_wedge_count_matches_closed_form(seed):
    g = _graph(seed, 500, 400, 6000)
    r = _vp(g.n_u, g.n_v, g.u, g.v, g.sign)
    assert r.wedges == _wedges_closed_form(g.n_u, g.n_v, g.u, g.v)
    assert r.expansions == g.m


def test_balanced_fraction_matches_iid_sign_law():
    # Statistical sanity, not a parity pin: with i.i.d. signs (negative with
    # probability q) a butterfly is balanced with probability (1+(1-2q)^4)/2.
    g = config_graph("powerlaw2m", scale=0.25)
    r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    assert abs(r.balanced / r.total - (1 + (1 - 2 * 0.25) ** 4) / 2) < 0.01


def test_build_once_count_split_over_pivots():
    """The oracle's separate build and count calls give the one-call counts,
    and Phase 5 over disjoint pivot sets adds up to the whole (Theorem 1: each
    butterfly is counted at exactly one pivot)."""
    from oracle import OracleGraph
    from synth import chung_lu_graph

    g = chung_lu_graph(900, 700, 9000, 2.1, 1.9, 0.4, seed=3)
    whole = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
    og = OracleGraph(g.n_u, g.n_v, g.u, g.v, g.sign)
    try:
        r = og.count(threads=3)
        assert (r.balanced, r.unbalanced, r.total, r.wedges) == (
            whole.balanced, whole.unbalanced, whole.total, whole.wedges)
        idx = np.arange(g.n_u + g.n_v)
        parts = [og.count(threads=1, pivots=idx[idx % 3 == k]) for k in range(3)]
        for f in ("balanced", "unbalanced", "total", "wedges", "expansions"):
            assert sum(getattr(p, f) for p in parts) == getattr(whole, f)
    finally:
        og.close()
