"""Brute-force butterfly classification (ORACLE, test infrastructure only).

Definition 1: a butterfly is a 4-cycle u - v - u' - v' with {u, u'} in U and
{v, v'} in V and all four edges present.  Definition 2: it is balanced when
the number of negative edges among the four is even, unbalanced otherwise.
This module loops over every pair of U times every pair of V; it is meant for
graphs of at most a few dozen vertices per side.
"""

from __future__ import annotations

from itertools import combinations


def _edge_map(u, v, sign):
    e = {}
    for a, b, s in zip(u, v, sign):
        e[(int(a), int(b))] = int(s)
    return e


def brute_counts(n_u, n_v, u, v, sign):
    """Return (balanced, unbalanced, total) by enumerating every 2x2 vertex set."""
    e = _edge_map(u, v, sign)
    bal = unb = 0
    for a, a2 in combinations(range(n_u), 2):
        for b, b2 in combinations(range(n_v), 2):
            quad = [(a, b), (a, b2), (a2, b), (a2, b2)]
            if not all(q in e for q in quad):
                continue
            negatives = sum(1 for q in quad if e[q] < 0)
            if negatives % 2 == 0:
                bal += 1
            else:
                unb += 1
    return bal, unb, bal + unb


def brute_per_vertex(n_u, n_v, u, v, sign):
    """Per vertex, the number of balanced / unbalanced butterflies containing it.

    Returns four lists: bal_u[n_u], bal_v[n_v], unb_u[n_u], unb_v[n_v].
    """
    e = _edge_map(u, v, sign)
    bal_u, bal_v = [0] * n_u, [0] * n_v
    unb_u, unb_v = [0] * n_u, [0] * n_v
    for a, a2 in combinations(range(n_u), 2):
        for b, b2 in combinations(range(n_v), 2):
            quad = [(a, b), (a, b2), (a2, b), (a2, b2)]
            if not all(q in e for q in quad):
                continue
            negatives = sum(1 for q in quad if e[q] < 0)
            tu, tv = (bal_u, bal_v) if negatives % 2 == 0 else (unb_u, unb_v)
            tu[a] += 1
            tu[a2] += 1
            tv[b] += 1
            tv[b2] += 1
    return bal_u, bal_v, unb_u, unb_v


def brute_per_edge(n_u, n_v, u, v, sign):
    """Per edge (in input order), the number of balanced and of unbalanced
    butterflies containing it.  Returns two lists: bal_e[m], unb_e[m]."""
    e = _edge_map(u, v, sign)
    bal = {k: 0 for k in e}
    unb = {k: 0 for k in e}
    for a, a2 in combinations(range(n_u), 2):
        for b, b2 in combinations(range(n_v), 2):
            quad = [(a, b), (a, b2), (a2, b), (a2, b2)]
            if not all(q in e for q in quad):
                continue
            cnt = bal if sum(1 for q in quad if e[q] < 0) % 2 == 0 else unb
            for q in quad:
                cnt[q] += 1
    keys = [(int(a), int(b)) for a, b in zip(u, v)]
    return [bal[k] for k in keys], [unb[k] for k in keys]


def edge_counts_at(n_u, n_v, u, v, sign, records):
    """Balanced and unbalanced butterflies through each given edge record,
    by Definitions 1-2 around that edge alone: for edge (a, b), every a' in
    N(b) minus a and b' in N(a) minus b closes a butterfly when (a', b') is
    an edge, balanced when the product of its four signs is positive.
    Works on large graphs for edges whose two degrees have a modest
    product.  Records must name distinct (u, v) pairs."""
    import numpy as np

    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    sg = np.asarray(sign, np.int64)
    key = u * n_v + v
    order = np.argsort(key, kind="stable")
    skey = key[order]
    ssign = sg[order]
    by_u = np.argsort(u, kind="stable")
    by_v = np.argsort(v, kind="stable")
    u_start = np.searchsorted(u[by_u], np.arange(n_u + 1))
    v_start = np.searchsorted(v[by_v], np.arange(n_v + 1))
    bal, unb = [], []
    for i in records:
        a, b, s0 = int(u[i]), int(v[i]), int(sg[i])
        ra = by_u[u_start[a]:u_start[a + 1]]   # edges (a, b')
        rb = by_v[v_start[b]:v_start[b + 1]]   # edges (a', b)
        ra = ra[v[ra] != b]
        rb = rb[u[rb] != a]
        if ra.size == 0 or rb.size == 0:
            bal.append(0)
            unb.append(0)
            continue
        k = u[rb][:, None] * n_v + v[ra][None, :]          # (a', b') candidates
        pos = np.minimum(np.searchsorted(skey, k), skey.size - 1)
        present = skey[pos] == k
        prod = s0 * sg[rb][:, None] * sg[ra][None, :] * ssign[pos]
        bal.append(int(np.count_nonzero(present & (prod > 0))))
        unb.append(int(np.count_nonzero(present & (prod < 0))))
    return bal, unb
