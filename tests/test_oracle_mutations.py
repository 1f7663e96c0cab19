"""Plant plausible mistakes in a private copy of the oracle's C source and
check that the pins catch each one (the shipped oracle is never modified)."""

import os
import subprocess

import numpy as np
import pytest

from oracle import brute_counts, pair_counts
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
    assert _pins_pass(_compile(src, str(tmp_path), "clean"))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    with open(_SRC) as f:
        src = f.read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    lib = _compile(src.replace(old, new), str(tmp_path), name)
    assert not _pins_pass(lib), f"planted mistake {name} went unnoticed"
