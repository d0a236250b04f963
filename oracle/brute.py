"""Brute force from the definitions, for tiny graphs (test infrastructure).

Everything here enumerates: butterflies as all 2x2 vertex quadruples
(Definition 2), k-bitrusses as greatest fixpoints of "delete every edge in
fewer than k butterflies of the current subgraph" (Definition 4), bitruss
numbers as the largest k whose k-bitruss keeps the edge (Definition 5).
`sequential_peel` is the one-edge-at-a-time peel of the baseline algorithm
(Algorithm 1), used to pin the level-synchronous oracle.
"""
from __future__ import annotations

import itertools

import numpy as np


def _edge_index(n_upper, n_lower, row_ptr, col):
    idx = -np.ones((n_upper, n_lower), dtype=np.int64)
    for u in range(n_upper):
        for e in range(int(row_ptr[u]), int(row_ptr[u + 1])):
            idx[u, int(col[e])] = e
    return idx


def butterflies(n_upper, n_lower, row_ptr, col):
    """Every butterfly as the sorted 4-tuple of its edge ids."""
    idx = _edge_index(n_upper, n_lower, row_ptr, col)
    out = []
    for u, w in itertools.combinations(range(n_upper), 2):
        for v, x in itertools.combinations(range(n_lower), 2):
            es = (idx[u, v], idx[u, x], idx[w, v], idx[w, x])
            if min(es) >= 0:
                out.append(tuple(sorted(int(e) for e in es)))
    return out


def support(n_upper, n_lower, row_ptr, col):
    """(per-edge support, total butterflies) by enumeration."""
    m = len(col)
    sup = np.zeros(m, dtype=np.int64)
    bf = butterflies(n_upper, n_lower, row_ptr, col)
    for b in bf:
        for e in b:
            sup[e] += 1
    return sup, len(bf)


def k_bitruss(bf, m, k, start=None):
    """Edge mask of the k-bitruss: greatest fixpoint from `start` (all edges)."""
    keep = np.ones(m, dtype=bool) if start is None else start.copy()
    while True:
        s = np.zeros(m, dtype=np.int64)
        for b in bf:
            if all(keep[e] for e in b):
                for e in b:
                    s[e] += 1
        drop = keep & (s < k)
        if not drop.any():
            return keep
        keep &= ~drop


def bitruss(n_upper, n_lower, row_ptr, col):
    """phi_e = max{k >= 0 : e in H_k}, with H_0 = G."""
    m = len(col)
    bf = butterflies(n_upper, n_lower, row_ptr, col)
    phi = np.zeros(m, dtype=np.int64)
    keep = np.ones(m, dtype=bool)
    k = 1
    while keep.any():
        keep = k_bitruss(bf, m, k, keep)   # H_k is inside H_{k-1}
        phi[keep] = k
        k += 1
    return phi


def sequential_peel(n_upper, n_lower, row_ptr, col):
    """Baseline peel: remove one minimum-support edge at a time.

    Its bitruss number is its current support; every other edge of each
    butterfly through it loses one butterfly if its support is larger.
    """
    m = len(col)
    bf = butterflies(n_upper, n_lower, row_ptr, col)
    s = np.zeros(m, dtype=np.int64)
    for b in bf:
        for e in b:
            s[e] += 1
    alive = np.ones(m, dtype=bool)
    by_edge = [[] for _ in range(m)]
    for i, b in enumerate(bf):
        for e in b:
            by_edge[e].append(i)
    live_bf = np.ones(len(bf), dtype=bool)
    phi = np.zeros(m, dtype=np.int64)
    for _ in range(m):
        cand = np.flatnonzero(alive)
        e = int(cand[np.argmin(s[cand])])
        phi[e] = s[e]
        for i in by_edge[e]:
            if not live_bf[i]:
                continue
            live_bf[i] = False
            for f in bf[i]:
                if f != e and s[f] > s[e]:
                    s[f] -= 1
        alive[e] = False
    return phi
