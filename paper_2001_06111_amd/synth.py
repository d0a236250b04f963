"""Seeded synthetic bipartite graphs shaped like the paper's workloads.

The paper evaluates on fifteen real bipartite graphs (Section VI, Table 2)
that are not available here.  This module draws stand-ins with the same
kind of shape: a uniform random graph for the small case and Chung-Lu
power-law graphs (expected-degree edge sampling) for the skewed cases,
plus the many-small-graphs pool and the Poisson request stream used by the
batched and served modes.

This module holds only input generation and CSR formatting.  It computes
nothing the decomposition computes; both the GPU path and the CPU oracle
take their inputs from here.

Graph format (shared by every consumer): upper-major CSR.
  row_ptr : int64[n_upper + 1], row_ptr[0] = 0, non-decreasing, row_ptr[-1] = m
  col     : int32[m], lower ids in [0, n_lower), strictly increasing per row
Edge e is CSR position e.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GENERATOR_VERSION = 1


@dataclasses.dataclass
class Graph:
    n_upper: int
    n_lower: int
    row_ptr: np.ndarray  # int64[n_upper + 1]
    col: np.ndarray      # int32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def edges(self):
        """(upper, lower) endpoint arrays, indexed by edge id."""
        u = np.repeat(np.arange(self.n_upper, dtype=np.int64),
                      np.diff(self.row_ptr))
        return u, self.col.astype(np.int64)


def from_edges(n_upper: int, n_lower: int, edges, name: str = "") -> Graph:
    """Build the canonical CSR from (upper, lower) pairs; duplicates rejected."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e[:, 0].min() < 0 or e[:, 0].max() >= n_upper
                   or e[:, 1].min() < 0 or e[:, 1].max() >= n_lower):
        raise ValueError("edge endpoint out of range")
    key = e[:, 0] * max(n_lower, 1) + e[:, 1]
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate edge: the edge set of a bipartite graph is a set")
    u = key // max(n_lower, 1)
    v = key % max(n_lower, 1)
    row_ptr = np.zeros(n_upper + 1, dtype=np.int64)
    np.cumsum(np.bincount(u, minlength=n_upper), out=row_ptr[1:])
    return Graph(n_upper, n_lower, row_ptr, v.astype(np.int32), name)


def _csr_from_keys(n_upper: int, n_lower: int, keys: np.ndarray, name: str) -> Graph:
    keys = np.sort(keys)
    u = keys // n_lower
    v = (keys % n_lower).astype(np.int32)
    row_ptr = np.zeros(n_upper + 1, dtype=np.int64)
    np.cumsum(np.bincount(u, minlength=n_upper), out=row_ptr[1:])
    return Graph(n_upper, n_lower, row_ptr, v, name)


def _first_distinct(draw, m: int, chunk: int) -> np.ndarray:
    """Keys of the first m distinct pairs of an endless seeded pair stream.

    `draw(k)` returns the next k keys of the stream.  The stream is consumed
    in fixed chunks, so the result depends only on the seed.
    """
    keys = np.empty(0, dtype=np.int64)
    for _ in range(4096):
        keys = np.concatenate([keys, draw(chunk)])
        uniq, first = np.unique(keys, return_index=True)
        if uniq.size >= m:
            first.sort()
            return keys[first[:m]]
        keys = keys[np.sort(first)]
    raise RuntimeError("could not draw enough distinct edges")


def uniform(n_upper: int, n_lower: int, m: int, seed: int, name: str = "") -> Graph:
    """Uniform pairs, first m distinct (the small plain workload)."""
    if m > n_upper * n_lower:
        raise ValueError("m exceeds the number of vertex pairs")
    rng = np.random.default_rng(seed)

    def draw(k):
        u = rng.integers(0, n_upper, size=k, dtype=np.int64)
        v = rng.integers(0, n_lower, size=k, dtype=np.int64)
        return u * n_lower + v

    keys = _first_distinct(draw, m, max(m, 1024))
    return _csr_from_keys(n_upper, n_lower, keys, name or f"uniform-{n_upper}x{n_lower}-m{m}-s{seed}")


def expected_degrees(n: int, m: int, s: float, cap: float) -> np.ndarray:
    """Expected-degree profile d_i = c (i+1)^(-1/(s-1)) with sum m, capped.

    s is the degree-distribution exponent.  Vertices above `cap` are set to
    `cap` and the excess is spread over the uncapped vertices in proportion
    to their weight, repeated until no uncapped vertex exceeds the cap.
    """
    if cap * n < m:
        raise ValueError("cap too small for the requested edge count")
    d = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (s - 1.0))
    d *= m / d.sum()
    capped = np.zeros(n, dtype=bool)
    for _ in range(10 * n + 10):
        over = (d > cap) & ~capped
        if not over.any():
            break
        capped |= over
        d[capped] = cap
        rest = m - cap * capped.sum()
        free = ~capped
        d[free] *= rest / d[free].sum()
    return d


def chung_lu(n_upper: int, n_lower: int, m: int, s_upper: float, s_lower: float,
             cap_upper: float, cap_lower: float, seed: int, name: str = "") -> Graph:
    """Chung-Lu bipartite graph by edge sampling; first m distinct pairs.

    Each side gets the capped expected-degree profile of `expected_degrees`,
    randomly permuted over vertex ids so that id is independent of degree.
    Endpoints are drawn independently with probability proportional to the
    expected degree.
    """
    if m > n_upper * n_lower:
        raise ValueError("m exceeds the number of vertex pairs")
    rng = np.random.default_rng(seed)
    du = expected_degrees(n_upper, m, s_upper, cap_upper)
    dl = expected_degrees(n_lower, m, s_lower, cap_lower)
    wu = np.empty_like(du)
    wl = np.empty_like(dl)
    wu[rng.permutation(n_upper)] = du
    wl[rng.permutation(n_lower)] = dl
    cu = np.cumsum(wu)
    cl = np.cumsum(wl)

    def draw(k):
        u = np.searchsorted(cu, rng.random(k) * cu[-1], side="right")
        v = np.searchsorted(cl, rng.random(k) * cl[-1], side="right")
        np.minimum(u, n_upper - 1, out=u)
        np.minimum(v, n_lower - 1, out=v)
        return u.astype(np.int64) * n_lower + v.astype(np.int64)

    keys = _first_distinct(draw, m, max(m, 1024))
    return _csr_from_keys(n_upper, n_lower, keys,
                          name or f"chunglu-{n_upper}x{n_lower}-m{m}-s{seed}")


# --- named workloads -------------------------------------------------------

def plain_uniform_10k() -> Graph:
    """1,000 x 1,500 uniform, 10,000 edges (seed 0)."""
    return uniform(1000, 1500, 10_000, 0, "uniform-1000x1500-m10k")


def plain_chunglu_5m() -> Graph:
    """200k x 500k Chung-Lu, 5M edges, exponents 2.1 / 2.5, cap 50k (seed 1)."""
    return chung_lu(200_000, 500_000, 5_000_000, 2.1, 2.5, 50_000, 50_000, 1,
                    "chunglu-200kx500k-m5M")


def plain_hub_20m() -> Graph:
    """100k x 2M Chung-Lu, 20M edges, exponents 1.8 / 2.3, cap 200k (seed 2)."""
    return chung_lu(100_000, 2_000_000, 20_000_000, 1.8, 2.3, 200_000, 200_000, 2,
                    "chunglu-100kx2M-m20M-hub")


def scaled_chunglu(m: int, seed: int = 7) -> Graph:
    """The 5M-edge Chung-Lu shape scaled down to m edges (same aspect ratio)."""
    f = m / 5_000_000
    nu = max(8, int(round(200_000 * f)))
    nl = max(8, int(round(500_000 * f)))
    cap = max(4.0, 50_000 * f)
    return chung_lu(nu, nl, m, 2.1, 2.5, cap, cap, seed, f"chunglu-scaled-m{m}-s{seed}")


BATCH_BASE_SEED = 3_000_000
BIG_BASE_SEED = 4_000_000
ARRIVAL_SEED = 4


def batch_graph(i: int) -> Graph:
    """Graph i of the many-small-graphs pool (seed 3,000,000 + i).

    |U|, |L| log-uniform in [50, 20000]; m log-uniform in [200, 200000],
    clamped to |U||L|/4 so that every draw is feasible and not near-complete;
    exponent 2.2 on both sides; a vertex's expected degree is bounded only
    by the size of the other side.
    """
    rng = np.random.default_rng(BATCH_BASE_SEED + i)
    nu = int(math.floor(math.exp(rng.uniform(math.log(50), math.log(20000)))))
    nl = int(math.floor(math.exp(rng.uniform(math.log(50), math.log(20000)))))
    m = int(math.floor(math.exp(rng.uniform(math.log(200), math.log(200_000)))))
    m = min(m, (nu * nl) // 4)
    sub = int(rng.integers(0, 2**31 - 1))
    return chung_lu(nu, nl, m, 2.2, 2.2, float(nl), float(nu), sub, f"batch-{i}")


def big_serving_graph(j: int) -> Graph:
    """Large request graph j: 50k x 200k, 2M edges, exponent 2.0 (seed 4,000,000 + j)."""
    return chung_lu(50_000, 200_000, 2_000_000, 2.0, 2.0, 200_000.0, 50_000.0,
                    BIG_BASE_SEED + j, f"big-{j}")


def serving_arrivals(rate: float = 200.0, duration: float = 60.0, p_small: float = 0.95,
                     n_small: int = 4096, n_big: int = 32, seed: int = ARRIVAL_SEED):
    """Poisson request stream: list of (arrival_time_s, kind, pool_index)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        if rng.random() < p_small:
            out.append((t, "small", int(rng.integers(0, n_small))))
        else:
            out.append((t, "big", int(rng.integers(0, n_big))))
    return out


def complete(a: int, b: int) -> Graph:
    """K_{a,b}."""
    return from_edges(a, b, [(i, j) for i in range(a) for j in range(b)], f"K{a},{b}")


def vertex_sample(g: Graph, frac: float, seed: int) -> Graph:
    """Induced subgraph on a random fraction of the vertices of each layer.

    Sampling protocol of the paper's scalability experiments (Section VI).
    Kept vertices are renumbered in id order.
    """
    rng = np.random.default_rng(seed)
    keep_u = np.sort(rng.permutation(g.n_upper)[: max(1, int(g.n_upper * frac))])
    keep_l = np.sort(rng.permutation(g.n_lower)[: max(1, int(g.n_lower * frac))])
    new_u = np.full(g.n_upper, -1, dtype=np.int64)
    new_l = np.full(g.n_lower, -1, dtype=np.int64)
    new_u[keep_u] = np.arange(keep_u.size)
    new_l[keep_l] = np.arange(keep_l.size)
    u, v = g.edges()
    sel = (new_u[u] >= 0) & (new_l[v] >= 0)
    keys = new_u[u[sel]] * keep_l.size + new_l[v[sel]]
    return _csr_from_keys(int(keep_u.size), int(keep_l.size), keys,
                          f"{g.name}-vs{frac:g}-s{seed}")
