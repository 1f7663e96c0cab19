"""Lemma 1 pair form of the signed butterfly count (ORACLE, test infrastructure only).

For two distinct vertices a, b on one side, every common neighbour x on the
other side closes a wedge a - x - b.  The wedge is symmetric when the edges
(a, x) and (b, x) carry the same sign and asymmetric otherwise (Definitions 5
and 6).  With p_ab symmetric and n_ab asymmetric wedges between a and b:

* Lemma 1: a balanced butterfly on {a, b} is two symmetric or two asymmetric
  wedges, so there are C(p_ab, 2) + C(n_ab, 2) of them;
* one symmetric and one asymmetric wedge give an odd number of negative
  edges, so p_ab * n_ab butterflies on {a, b} are unbalanced;
* every butterfly has exactly one pair on each side, so summing over the
  pairs of either side counts each butterfly once.

``dense`` forms p and n with exact integer matrix products over the signed
adjacency; ``sparse`` walks, for every vertex x, all pairs of its neighbours.
"""

from __future__ import annotations

from collections import defaultdict
from itertools import combinations

import numpy as np


def _c2(x):
    return x * (x - 1) // 2


def _sides(n_u, n_v, u, v, sign, pair_side):
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    s = np.asarray(sign, dtype=np.int64)
    if pair_side == "u":
        return n_u, n_v, u, v, s
    return n_v, n_u, v, u, s


def pair_pn_dense(n_u, n_v, u, v, sign, pair_side="u"):
    """Matrices P, N (int64, n_pair x n_pair) of symmetric / asymmetric wedge
    counts between every two vertices of the pair side (diagonal meaningless)."""
    n_p, n_m, a, x, s = _sides(n_u, n_v, u, v, sign, pair_side)
    # 0/1 indicator matrices; float64 products of them are exact integers
    # (every entry is at most n_m, far below 2**53), then taken to int64.
    pos = np.zeros((n_p, n_m), dtype=np.float64)
    neg = np.zeros((n_p, n_m), dtype=np.float64)
    pos[a[s > 0], x[s > 0]] = 1.0
    neg[a[s < 0], x[s < 0]] = 1.0
    P = pos @ pos.T + neg @ neg.T
    N = pos @ neg.T + neg @ pos.T
    assert n_m < 2**53
    return np.rint(P).astype(np.int64), np.rint(N).astype(np.int64)


def pair_counts(n_u, n_v, u, v, sign, pair_side="u", method="dense"):
    """Return (balanced, unbalanced, total) as Python ints."""
    if method == "dense":
        P, N = pair_pn_dense(n_u, n_v, u, v, sign, pair_side)
        iu = np.triu_indices(P.shape[0], k=1)
        p, n = P[iu], N[iu]
        bal = int((_c2(p) + _c2(n)).sum())
        unb = int((p * n).sum())
        tot = int(_c2(p + n).sum())
        return bal, unb, tot
    pn = _pair_dict(n_u, n_v, u, v, sign, pair_side)
    bal = unb = tot = 0
    for p, n in pn.values():
        bal += _c2(p) + _c2(n)
        unb += p * n
        tot += _c2(p + n)
    return bal, unb, tot


def _adjacency(n_p, n_m, a, x, s):
    nbrs = [[] for _ in range(n_m)]
    for ai, xi, si in zip(a.tolist(), x.tolist(), s.tolist()):
        nbrs[xi].append((ai, si))
    return nbrs


def _pair_dict(n_u, n_v, u, v, sign, pair_side):
    n_p, n_m, a, x, s = _sides(n_u, n_v, u, v, sign, pair_side)
    pn = defaultdict(lambda: [0, 0])
    for lst in _adjacency(n_p, n_m, a, x, s):
        for (a1, s1), (a2, s2) in combinations(sorted(lst), 2):
            pn[(a1, a2)][0 if s1 == s2 else 1] += 1
    return pn


def pair_per_vertex(n_u, n_v, u, v, sign):
    """Per vertex, balanced and unbalanced butterflies containing it, from the
    pair form with pairs on U.  Returns int64 arrays bal_u, bal_v, unb_u, unb_v.

    A pair {a, b} lies in C(p,2) + C(n,2) balanced and p * n unbalanced
    butterflies.  A common neighbour x of a symmetric wedge a - x - b lies in
    p - 1 of the balanced ones (paired with each other symmetric wedge) and in
    n unbalanced ones; for an asymmetric wedge the roles of p and n swap.
    """
    n_p, n_m, a, x, s = _sides(n_u, n_v, u, v, sign, "u")
    pn = _pair_dict(n_u, n_v, u, v, sign, "u")
    bal_u = np.zeros(n_u, np.int64)
    unb_u = np.zeros(n_u, np.int64)
    bal_v = np.zeros(n_v, np.int64)
    unb_v = np.zeros(n_v, np.int64)
    for (a1, a2), (p, n) in pn.items():
        c = _c2(p) + _c2(n)
        bal_u[a1] += c
        bal_u[a2] += c
        unb_u[a1] += p * n
        unb_u[a2] += p * n
    for xi, lst in enumerate(_adjacency(n_p, n_m, a, x, s)):
        for (a1, s1), (a2, s2) in combinations(sorted(lst), 2):
            p, n = pn[(a1, a2)]
            if s1 == s2:
                bal_v[xi] += p - 1
                unb_v[xi] += n
            else:
                bal_v[xi] += n - 1
                unb_v[xi] += p
    return bal_u, bal_v, unb_u, unb_v
