"""Small hand-built graphs for pins and parity cases (input construction only)."""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

from paper_2001_06111_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def worked_example(with_grey: bool = True):
    """The paper's running example; edge ids follow e0..e8, grey edges last."""
    fx = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    named = [tuple(fx["named_edges"][f"e{i}"]) for i in range(9)]
    edges = named + ([tuple(e) for e in fx["grey_edges"]] if with_grey else [])
    g = synth.from_edges(fx["n_upper"], fx["n_lower"], edges, "worked-example")
    # CSR order (upper-major, lower ascending) coincides with e0..e8 then grey.
    u, v = g.edges()
    assert [tuple(p) for p in zip(u.tolist(), v.tolist())] == sorted(edges)
    pos = {p: i for i, p in enumerate(zip(u.tolist(), v.tolist()))}
    names = {f"e{i}": pos[named[i]] for i in range(9)}
    if with_grey:
        names["grey0"] = pos[tuple(fx["grey_edges"][0])]
        names["grey1"] = pos[tuple(fx["grey_edges"][1])]
    return g, names, fx


def fig2a():
    """Section I observation graph: 4,002 vertices, one butterfly [u0,v0,u1,v1].

    u0 - v0, v1; u1 - v0..v1000; v1 - u0..u1000; u2 - v1001..v2000;
    v2 - u1001..u2000.
    """
    e = {(0, 0), (0, 1)}
    e |= {(1, j) for j in range(0, 1001)}
    e |= {(i, 1) for i in range(0, 1001)}
    e |= {(2, j) for j in range(1001, 2001)}
    e |= {(i, 2) for i in range(1001, 2001)}
    return synth.from_edges(2001, 2001, sorted(e), "fig2a")


def k2_1001():
    """Section I: the (2,1001)-biclique; e_i = (u0, v_i), e_{i+1001} = (u1, v_i)."""
    return synth.complete(2, 1001)


def cycle(k: int):
    """Even cycle C_{2k}: u_i - v_i - u_{i+1}."""
    e = [(i, i) for i in range(k)] + [((i + 1) % k, i) for i in range(k)]
    return synth.from_edges(k, k, sorted(set(e)), f"C{2*k}")


def star(leaves: int, center_upper: bool = True):
    if center_upper:
        return synth.from_edges(1, leaves, [(0, j) for j in range(leaves)], "star")
    return synth.from_edges(leaves, 1, [(i, 0) for i in range(leaves)], "star")


def random_forest(nu: int, nl: int, seed: int):
    """A random bipartite forest: each new vertex attaches to one earlier vertex."""
    rng = np.random.default_rng(seed)
    order = [("u", i) for i in range(nu)] + [("l", j) for j in range(nl)]
    rng.shuffle(order)
    edges = []
    seen_u, seen_l = [], []
    for side, i in order:
        other = seen_l if side == "u" else seen_u
        if other and rng.random() < 0.8:
            j = other[int(rng.integers(0, len(other)))]
            edges.append((i, j) if side == "u" else (j, i))
        (seen_u if side == "u" else seen_l).append(i)
    return synth.from_edges(nu, nl, edges, "forest")


def all_graphs(nu: int, nl: int):
    """Every bipartite graph on nu x nl labelled vertices."""
    pairs = [(i, j) for i in range(nu) for j in range(nl)]
    for mask in range(1 << len(pairs)):
        yield synth.from_edges(nu, nl, [p for b, p in enumerate(pairs) if mask >> b & 1])


def random_dense(nu: int, nl: int, p: float, seed: int):
    rng = np.random.default_rng(seed)
    pairs = [(i, j) for i in range(nu) for j in range(nl) if rng.random() < p]
    return synth.from_edges(nu, nl, pairs, f"dense-{nu}x{nl}-{seed}")


def disjoint_union(a, b):
    ua, va = a.edges()
    ub, vb = b.edges()
    e = list(zip(ua.tolist(), va.tolist())) + list(zip((ub + a.n_upper).tolist(), (vb + a.n_lower).tolist()))
    return synth.from_edges(a.n_upper + b.n_upper, a.n_lower + b.n_lower, e, "union")


def relabel(g, seed: int):
    """Permute ids inside each layer; returns (graph, old edge id -> new edge id)."""
    rng = np.random.default_rng(seed)
    pu = rng.permutation(g.n_upper)
    pl = rng.permutation(g.n_lower)
    u, v = g.edges()
    nu_, nv_ = pu[u], pl[v]
    h = synth.from_edges(g.n_upper, g.n_lower, list(zip(nu_.tolist(), nv_.tolist())), "relabel")
    key_new = nu_ * g.n_lower + nv_
    hu, hv = h.edges()
    hkey = hu * g.n_lower + hv
    return h, np.searchsorted(hkey, key_new)


def swap_layers(g):
    """Exchange the upper and lower layers; returns (graph, old id -> new id)."""
    u, v = g.edges()
    h = synth.from_edges(g.n_lower, g.n_upper, list(zip(v.tolist(), u.tolist())), "swap")
    hu, hv = h.edges()
    hkey = hu * g.n_upper + hv
    return h, np.searchsorted(hkey, v * g.n_upper + u)


def induced_edges(g, mask):
    """Subgraph on the edges where mask is true; returns (graph, new -> old id)."""
    u, v = g.edges()
    sel = np.flatnonzero(mask)
    h = synth.from_edges(g.n_upper, g.n_lower, list(zip(u[sel].tolist(), v[sel].tolist())), "sub")
    return h, sel  # from_edges keeps upper-major order, the same order as sel
