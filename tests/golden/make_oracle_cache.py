"""Write tests/golden/oracle_cache.json: CPU-oracle counts of the full-size
synthetic workloads, too slow to recompute inside every GPU test run.

Every value comes from oracle.vp_counts (Algorithm 1 Phase 5 in plain C) on
the graph that synth.config_graph generates for the named workload.

    python tests/golden/make_oracle_cache.py [name ...]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import vp_counts  # noqa: E402
from synth import config_graph  # noqa: E402

OUT = os.path.join(HERE, "oracle_cache.json")


def main(names):
    cache = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            cache = json.load(f)
    for name in names:
        g = config_graph(name)
        t = time.time()
        r = vp_counts(g.n_u, g.n_v, g.u, g.v, g.sign)
        cache[name] = dict(n_u=g.n_u, n_v=g.n_v, m=g.m, balanced=r.balanced,
                           unbalanced=r.unbalanced, total=r.total, wedges=r.wedges,
                           expansions=r.expansions)
        print(name, cache[name], f"{time.time() - t:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["tiny", "powerlaw2m", "skewed50m"])
