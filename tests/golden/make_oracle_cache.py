"""Write tests/golden/oracle_cache.json: CPU-oracle counts of the full-size
synthetic workloads, too slow to recompute inside every GPU test run.

Every value comes from oracle.vp_counts (Algorithm 1 Phase 5 in plain C) on
the graph that synth.config_graph generates for the named workload.  With
``--local`` the named workloads also get the oracle's per-vertex and
per-edge counts (the butterflies containing each vertex or edge, the
measures of the paper's Section I applications): a SHA-256 digest of each
int64 array (little-endian, U then V for vertices, input-record order for
edges) and the explicit values at sampled edges, chosen among the edges
with the largest degree products and among edges at a vertex whose degree
times the other side's largest degree reaches 2^32 (the edges whose
butterfly counts can exceed 32 bits).

    python tests/golden/make_oracle_cache.py [--local] [name ...]
"""

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import vp_counts  # noqa: E402
from synth import config_graph  # noqa: E402

OUT = os.path.join(HERE, "oracle_cache.json")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def sample_edges(g, k_top=40, k_wide=40, seed=11):
    """Edge records to store explicitly: the ``k_top`` largest degree
    products, and ``k_wide`` drawn at random among edges at a vertex whose
    degree times the other side's largest degree reaches 2^32."""
    deg_u = np.bincount(g.u, minlength=g.n_u).astype(np.int64)
    deg_v = np.bincount(g.v, minlength=g.n_v).astype(np.int64)
    du, dv = deg_u[g.u], deg_v[g.v]
    prod = du * dv
    top = np.argsort(-prod, kind="stable")[:k_top]
    wide = np.flatnonzero((du * int(deg_v.max()) >= 1 << 32) | (dv * int(deg_u.max()) >= 1 << 32))
    wide = np.setdiff1d(wide, top)
    rng = np.random.default_rng(seed)
    pick = rng.choice(wide, min(k_wide, wide.shape[0]), replace=False) if wide.shape[0] else wide
    return np.sort(np.concatenate([top, pick])).astype(np.int64), int(wide.shape[0])


def main(args):
    local = "--local" in args
    names = [a for a in args if not a.startswith("--")]
    cache = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            cache = json.load(f)
    for name in names or ["tiny", "powerlaw2m", "skewed50m"]:
        g = config_graph(name)
        t = time.time()
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign, per_vertex=local, per_edge=local)
        entry = cache.get(name, {})
        entry.update(n_u=g.n_u, n_v=g.n_v, m=g.m, balanced=r.balanced,
                     unbalanced=r.unbalanced, total=r.total, wedges=r.wedges,
                     expansions=r.expansions)
        if local:
            edges, n_wide = sample_edges(g)
            entry["local"] = dict(
                sha256={k: digest(getattr(r, k)) for k in
                        ("bal_u", "bal_v", "unb_u", "unb_v", "bal_e", "unb_e")},
                edges=[int(e) for e in edges],
                bal_e=[int(r.bal_e[e]) for e in edges],
                unb_e=[int(r.unb_e[e]) for e in edges],
                wide_edges=n_wide)
        cache[name] = entry
        print(name, {k: v for k, v in entry.items() if k != "local"},
              f"{time.time() - t:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
