"""The BE-Index from its definition (test infrastructure).

Section IV of the paper: the priority of a vertex orders by degree, ties
by id (Definition 6), and every upper id exceeds every lower id (Section
II).  A maximal priority-obeyed bloom (Definition 7) has its
highest-priority vertex x in its two-vertex layer {x, z}; maximality makes
its other layer the set M = {y in N(x) & N(z) : p(y) < p(x)}, and it is a
bloom only if |M| >= 2.  Its wedges are the pairs of edges (x,y), (z,y) for
y in M; the two edges of a pair are each other's twin (Definition 8).
Edge ids are CSR positions.
"""
from __future__ import annotations

import numpy as np


def priority_keys(n_upper, n_lower, row_ptr, col):
    """(degree, id) keys: lower j has id j, upper i has id n_lower + i.

    Returned as one int64 per vertex, vertex index = id; comparing keys
    compares priorities.
    """
    du = np.diff(np.asarray(row_ptr, dtype=np.int64))
    dl = np.bincount(np.asarray(col, dtype=np.int64), minlength=n_lower)
    deg = np.concatenate([dl, du]).astype(np.int64)
    gid = np.arange(n_lower + n_upper, dtype=np.int64)
    return deg * (n_lower + n_upper) + gid


def _neighbours(n_upper, n_lower, row_ptr, col):
    """Neighbour id lists (by global id) and edge-id lookup."""
    nbr = [[] for _ in range(n_lower + n_upper)]
    eid = {}
    for u in range(n_upper):
        for e in range(int(row_ptr[u]), int(row_ptr[u + 1])):
            v = int(col[e])
            gu = n_lower + u
            nbr[gu].append(v)
            nbr[v].append(gu)
            eid[(gu, v)] = e
            eid[(v, gu)] = e
    return nbr, eid


def blooms(n_upper, n_lower, row_ptr, col):
    """All maximal priority-obeyed blooms, canonically ordered.

    Each bloom is (x, z, ((e_xy, e_zy), ...)) with x the highest-priority
    vertex, z the other dominant-layer vertex (global ids), and the wedge
    edge pairs sorted by y.  Quadratic in the layer sizes: tiny graphs only.
    """
    key = priority_keys(n_upper, n_lower, row_ptr, col)
    nbr, eid = _neighbours(n_upper, n_lower, row_ptr, col)
    sets = [set(a) for a in nbr]
    out = []
    for layer in (range(n_lower), range(n_lower, n_lower + n_upper)):
        for x in layer:
            for z in layer:
                if z == x or key[z] >= key[x]:
                    continue
                M = sorted(y for y in sets[x] & sets[z] if key[y] < key[x])
                if len(M) >= 2:
                    out.append((x, z, tuple((eid[(x, y)], eid[(z, y)]) for y in M)))
    out.sort()
    return out


def blooms_at(x, n_upper, n_lower, row_ptr, col, key=None, nbr=None):
    """Blooms whose highest-priority vertex is x (global id), canonical order.

    For sampled checks on graphs too large for `blooms`: collects
    M(x, z) = {y in N(x) : p(y) < p(x), z in N(y), p(z) < p(x)} for every z.
    """
    if key is None:
        key = priority_keys(n_upper, n_lower, row_ptr, col)
    if nbr is None:
        nbr, _ = _neighbours(n_upper, n_lower, row_ptr, col)
    M = {}
    for y in nbr[x]:
        if key[y] >= key[x]:
            continue
        for z in nbr[y]:
            if z != x and key[z] < key[x]:
                M.setdefault(z, []).append(y)
    return sorted((x, z, tuple(sorted(ys))) for z, ys in M.items() if len(ys) >= 2)
