"""Connected components of a k-bitruss, from the definitions (test infrastructure).

H_k is the set of edges whose bitruss number is at least k (Definitions 4-5);
its components are found by breadth-first search over the vertices that these
edges join.  Components are numbered 0, 1, ... in order of their smallest edge
id; edges outside H_k get -1.  Shares no code with the GPU path.
"""
from collections import deque

import numpy as np


def bitruss_components(n_upper, n_lower, row_ptr, col, phi, k):
    """(comp int32[m], number of components) for H_k = {e : phi[e] >= k}."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    phi = np.asarray(phi)
    m = len(col)
    upper = np.repeat(np.arange(n_upper, dtype=np.int64), np.diff(row_ptr))
    # vertex v: lower j -> j, upper i -> n_lower + i; adjacency lists of H_k edges
    adj = [[] for _ in range(n_upper + n_lower)]
    for e in range(m):
        if phi[e] >= k:
            a, b = n_lower + int(upper[e]), int(col[e])
            adj[a].append((b, e))
            adj[b].append((a, e))
    comp = np.full(m, -1, dtype=np.int32)
    count = 0
    for e0 in range(m):  # increasing edge id: the first unlabelled edge opens a component
        if phi[e0] < k or comp[e0] >= 0:
            continue
        start = n_lower + int(upper[e0])
        seen = {start}
        queue = deque([start])
        while queue:
            v = queue.popleft()
            for w, e in adj[v]:
                comp[e] = count
                if w not in seen:
                    seen.add(w)
                    queue.append(w)
        count += 1
    return comp, count
