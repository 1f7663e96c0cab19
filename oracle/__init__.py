"""CPU oracle for signed butterfly counting -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the GPU library and the library never
calls it.  Three tiers, each written from the paper's text:

* ``brute``: Definitions 1-2 verbatim -- every pair {u, u'} of U times every
  pair {v, v'} of V, all four edges present, balanced iff the number of
  negative edges is even.  For graphs with a few dozen vertices per side.
* ``pairs``: the Lemma 1 form -- per same-side vertex pair, the number of
  common neighbours reached by two equal-sign edges (p) and by two
  different-sign edges (n); balanced = sum C(p,2) + C(n,2), unbalanced =
  sum p * n.  Dense matrix products for small graphs, sparse loops otherwise.
* ``vp``: Algorithm 1 Phase 5 (vertex priority, Definition 3) in plain C with
  POSIX threads (``vp.c``); also the timed CPU baseline.

Every count is an exact Python / int64 integer.
"""

from .brute import brute_counts, brute_per_edge, brute_per_vertex, edge_counts_at  # noqa: F401
from .pairs import pair_counts, pair_per_vertex  # noqa: F401
from .vp import OracleGraph, vp_counts, build as build_vp  # noqa: F401
