"""Plant plausible mistakes in a private copy of the oracle's C source and
check that the pins catch each one (the shipped oracle is never modified)."""

import os
import subprocess

import numpy as np
import pytest

from oracle import brute_counts, brute_per_edge, brute_per_vertex, pair_counts
from oracle.vp import _SRC, vp_counts
from synth import uniform_graph

from golden_io import load
from test_oracle_pins import _wedges_closed_form

MUTATIONS = {
    "no_mid_filter": ("      if (!higher(J, u, v)) continue;\n      c.expansions",
                      "      c.expansions"),
    "endpoint_filter_flipped": ("        if (!higher(J, u, w)) continue;\n        c.wedges",
                                "        if (higher(J, u, w) || w == u) continue;\n        c.wedges"),
    "pivot_edge_sign_ignored": ("if (J->adj_sign[a] == J->adj_sign[b])\n          B1[w] += 1;",
                                "if (J->adj_sign[b] > 0)\n          B1[w] += 1;"),
    "choose2_off_by_one": ("return x * (x - 1) / 2;", "return x * (x + 1) / 2;"),
    "unbalanced_dropped_factor": ("int64_t unb = (int64_t)B1[w] * B2[w];",
                                  "int64_t unb = (int64_t)B1[w];"),
    "degree_order_reversed": ("return J->deg[a] > J->deg[b];", "return J->deg[a] < J->deg[b];"),
    "no_reset": ("      B1[touched[t]] = 0;\n      B2[touched[t]] = 0;", ""),
}

# mistakes in the per-vertex / per-edge credit pass
CREDIT_MUTATIONS = {
    "mid_credit_keeps_self": ("            bw = B1[w] - 1;", "            bw = B1[w];"),
    "asym_roles_not_swapped": ("            bw = B2[w] - 1;\n            uw = B1[w];",
                               "            bw = B1[w] - 1;\n            uw = B2[w];"),
    "edge_credit_one_end": ("            add_vertex(J->bal_edge, J->adj_eid[b], bw);\n", ""),
    "unb_edge_takes_bal": ("            add_vertex(J->unb_edge, J->adj_eid[a], uw);",
                           "            add_vertex(J->unb_edge, J->adj_eid[a], bw);"),
    "pivot_credit_dropped": ("      if (J->bal_vertex) add_vertex(J->bal_vertex, u, pivot_bal);\n", ""),
}


def _pins_pass(lib):
    # the paper's worked example, pivot attribution included
    (fx,) = load("k22_example.txt")
    n_u, n_v, u, v, s = fx.arrays()
    ids = np.array([int(k) for k in fx.left] + [int(k) for k in fx.right], np.int64)
    r = vp_counts(n_u, n_v, u, v, s, ids=ids, per_pivot=True, threads=1, lib_path=lib)
    if (r.balanced, r.unbalanced, r.total) != (1, 0, 1) or r.per_pivot_bal[fx.vertex("R8")] != 1:
        return False
    # brute force and the pair form on random small graphs
    for seed in range(60):
        rng = np.random.default_rng(seed)
        g = uniform_graph(int(rng.integers(2, 9)), int(rng.integers(2, 9)),
                          int(rng.integers(4, 40)), 0.4, seed=seed)
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, threads=2, lib_path=lib)
        got = (r.balanced, r.unbalanced, r.total)
        if got != brute_counts(g.n_u, g.n_v, g.u, g.v, g.sign):
            return False
        if got != pair_counts(g.n_u, g.n_v, g.u, g.v, g.sign):
            return False
        # the order changes only who counts a butterfly and how many wedges
        # are walked (Theorem 1); the walked wedges have a closed form
        if r.wedges != _wedges_closed_form(g.n_u, g.n_v, g.u, g.v):
            return False
    return True


def _credit_pins_pass(lib):
    # brute force per vertex and per edge on random small graphs, and the
    # paper's figure (balanced butterflies per vertex and per edge)
    (fx,) = load("fig_comparison.txt")
    n_u, n_v, u, v, s = fx.arrays()
    r = vp_counts(n_u, n_v, u, v, s, per_vertex=True, per_edge=True, threads=1, lib_path=lib)
    if list(r.bal_u) != [2, 2, 3, 3, 2, 2, 0]:
        return False
    for seed in range(40):
        rng = np.random.default_rng(seed)
        g = uniform_graph(int(rng.integers(2, 9)), int(rng.integers(2, 9)),
                          int(rng.integers(4, 40)), 0.4, seed=seed)
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=True, per_edge=True,
                      threads=2, lib_path=lib)
        bvx = brute_per_vertex(g.n_u, g.n_v, g.u, g.v, g.sign)
        for a, b in zip(bvx, (r.bal_u, r.bal_v, r.unb_u, r.unb_v)):
            if list(a) != list(b):
                return False
        be, ue = brute_per_edge(g.n_u, g.n_v, g.u, g.v, g.sign)
        if list(r.bal_e) != be or list(r.unb_e) != ue:
            return False
    return True


def _compile(src_text, out_dir, name):
    c = os.path.join(out_dir, f"{name}.c")
    so = os.path.join(out_dir, f"{name}.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-shared", "-fPIC", "-pthread", "-o", so, c])
    return so


def test_unmutated_copy_passes(tmp_path):
    with open(_SRC) as f:
        src = f.read()
    lib = _compile(src, str(tmp_path), "clean")
    assert _pins_pass(lib) and _credit_pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    with open(_SRC) as f:
        src = f.read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    lib = _compile(src.replace(old, new), str(tmp_path), name)
    assert not _pins_pass(lib), f"planted mistake {name} went unnoticed"


@pytest.mark.parametrize("name", sorted(CREDIT_MUTATIONS))
def test_credit_mutation_is_caught(name, tmp_path):
    with open(_SRC) as f:
        src = f.read()
    old, new = CREDIT_MUTATIONS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    lib = _compile(src.replace(old, new), str(tmp_path), name)
    assert not _credit_pins_pass(lib), f"planted mistake {name} went unnoticed"
