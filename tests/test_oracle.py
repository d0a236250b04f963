"""Pins for the CPU oracle: printed values, closed forms, brute force, invariants.

Everything here runs on the CPU.  The oracle is checked against things other
than itself: values the paper prints for its running example, closed forms,
exhaustive brute force of the definitions on tiny graphs, and invariants
that hold at any size.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute, index_def
from paper_2001_06111_amd import synth
from tests import graphs


def osup(g, **kw):
    return oracle.support(g.n_upper, g.n_lower, g.row_ptr, g.col, **kw)


def ophi(g, **kw):
    return oracle.bitruss(g.n_upper, g.n_lower, g.row_ptr, g.col, **kw)


# --- the paper's worked example -------------------------------------------

@pytest.mark.parametrize("with_grey", [True, False])
def test_worked_example_printed_values(with_grey):
    g, nm, fx = graphs.worked_example(with_grey)
    sup, bf, pairs = osup(g)
    for name, val in fx["support"].items():
        assert sup[nm[name]] == val, name
    phi, st = ophi(g)
    for i in range(9):
        assert phi[nm[f"e{i}"]] == fx["phi"][f"e{i}"]
    if with_grey:
        assert sup[nm["grey0"]] == 0 and sup[nm["grey1"]] == 0
        assert phi[nm["grey0"]] == fx["phi"]["grey"] and phi[nm["grey1"]] == fx["phi"]["grey"]
    # the 3-bloom H2 holds 3 butterflies, the 2-bloom one: 4 in all
    assert bf == pairs == fx["bloom_B0_butterflies"] + 1
    assert st["destroyed"] == bf


def test_worked_example_remove_e6():
    """Deleting e6 lowers e5 by (2-1) and leaves e7, e8 with no butterfly."""
    g, nm, fx = graphs.worked_example(False)
    keep = np.ones(g.m, dtype=bool)
    keep[nm["e6"]] = False
    h, old = graphs.induced_edges(g, keep)
    sup, _, _ = osup(h)
    new_of = {int(o): i for i, o in enumerate(old)}
    assert sup[new_of[nm["e5"]]] == fx["support_e5_after_removing_e6"]
    assert sup[new_of[nm["e7"]]] == 0 and sup[new_of[nm["e8"]]] == 0


def test_worked_example_index_9edge():
    g, nm, fx = graphs.worked_example(False)
    bl = index_def.blooms(g.n_upper, g.n_lower, g.row_ptr, g.col)
    nl = g.n_lower
    name = {j: f"v{j}" for j in range(nl)}
    name.update({nl + i: f"u{i}" for i in range(g.n_upper)})
    got = {}
    for x, z, wedges in bl:
        got[(name[x], name[z])] = wedges
    b0 = fx["index_9edge"]["B0"]
    b1 = fx["index_9edge"]["B1"]
    assert set(got) == {tuple(b0["dominant"]), tuple(b1["dominant"])}
    assert len(got[tuple(b0["dominant"])]) == len(b0["other"])
    assert len(got[tuple(b1["dominant"])]) == len(b1["other"])
    # twin of e0 in B0: the pair holding e0 holds e1
    pair = [p for p in got[tuple(b0["dominant"])] if nm["e0"] in p][0]
    assert set(pair) == {nm["e0"], nm[fx["index_9edge"]["twin_e0_in_B0"]]}


def test_worked_example_index_11edge_tie():
    """With the grey edges d(u2) = d(v1) = 4 and the larger id (u2) wins the
    tie, so the index is four 2-blooms; the butterfly total is unchanged."""
    g, nm, fx = graphs.worked_example(True)
    bl = index_def.blooms(g.n_upper, g.n_lower, g.row_ptr, g.col)
    assert sorted(len(w) for _, _, w in bl) == [2, 2, 2, 2]
    assert sum(math.comb(len(w), 2) for _, _, w in bl) == 4


def test_fig2a_one_butterfly():
    g = graphs.fig2a()
    assert g.n_upper + g.n_lower == 4002 and g.m == 4002
    sup, bf, pairs = osup(g)
    assert bf == 1 and pairs == 1
    u, v = g.edges()
    in_bf = {(0, 0), (0, 1), (1, 0), (1, 1)}
    mask = np.array([(a, b) in in_bf for a, b in zip(u.tolist(), v.tolist())])
    assert np.all(sup[mask] == 1) and np.all(sup[~mask] == 0)
    phi, _ = ophi(g)
    assert np.array_equal(phi, mask.astype(np.int64))


def test_k2_1001():
    g = graphs.k2_1001()
    sup, bf, pairs = osup(g)
    assert bf == pairs == 1001 * 1000 // 2
    assert np.all(sup == 1000)
    phi, _ = ophi(g)
    assert np.all(phi == 1000)
    bl = index_def.blooms(g.n_upper, g.n_lower, g.row_ptr, g.col)
    assert len(bl) == 1 and len(bl[0][2]) == 1001
    for ea, eb in bl[0][2]:      # twins: e_i <-> e_{i+1001}
        assert abs(ea - eb) == 1001


# --- closed forms ----------------------------------------------------------

@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (2, 2), (2, 7), (3, 3), (4, 6), (7, 5), (12, 9)])
def test_complete_bipartite(a, b):
    g = synth.complete(a, b)
    sup, bf, pairs = osup(g)
    assert np.all(sup == (a - 1) * (b - 1))
    assert bf == pairs == math.comb(a, 2) * math.comb(b, 2)
    phi, _ = ophi(g)
    assert np.all(phi == (a - 1) * (b - 1))


def test_zero_butterfly_families():
    cases = [graphs.star(9), graphs.star(7, False), graphs.cycle(3), graphs.cycle(5),
             graphs.cycle(8)] + [graphs.random_forest(30, 40, s) for s in range(5)]
    for g in cases:
        sup, bf, _ = osup(g)
        assert bf == 0 and not sup.any()
        phi, _ = ophi(g)
        assert not phi.any()
    g = graphs.cycle(2)                  # C4 is a butterfly
    sup, bf, _ = osup(g)
    assert bf == 1 and np.all(sup == 1)


def test_empty_graph():
    g = synth.from_edges(3, 4, [])
    sup, bf, _ = osup(g)
    assert sup.size == 0 and bf == 0
    phi, st = ophi(g)
    assert phi.size == 0 and st["rounds"] == 0


# --- exhaustive brute force -----------------------------------------------

def _check_against_brute(g):
    bs, bb = brute.support(g.n_upper, g.n_lower, g.row_ptr, g.col)
    for orient in (1, 2):
        sup, bf, pairs = osup(g, orientation=orient)
        assert np.array_equal(sup, bs) and bf == bb and pairs == bb
    phi, st = ophi(g)
    assert np.array_equal(phi, brute.bitruss(g.n_upper, g.n_lower, g.row_ptr, g.col))
    assert np.array_equal(phi, brute.sequential_peel(g.n_upper, g.n_lower, g.row_ptr, g.col))
    assert st["destroyed"] == bb


@pytest.mark.parametrize("nu,nl", [(2, 2), (2, 3), (3, 3), (3, 4)])
def test_exhaustive_small(nu, nl):
    for g in graphs.all_graphs(nu, nl):
        _check_against_brute(g)


@pytest.mark.parametrize("seed", range(30))
def test_random_small_vs_brute(seed):
    rng = np.random.default_rng(seed)
    nu, nl = int(rng.integers(3, 11)), int(rng.integers(3, 11))
    g = graphs.random_dense(nu, nl, float(rng.uniform(0.3, 0.9)), seed)
    _check_against_brute(g)


# --- invariants at larger sizes --------------------------------------------

@pytest.fixture(scope="module")
def medium():
    return [synth.scaled_chunglu(20_000, seed=11), synth.uniform(300, 400, 6000, 5),
            graphs.random_dense(40, 50, 0.5, 3)]


def test_support_invariants(medium):
    for g in medium:
        sup, bf, pairs = osup(g)
        assert sup.sum() == 4 * bf and bf == pairs
        u, v = g.edges()
        du = np.diff(g.row_ptr)
        dl = np.bincount(g.col, minlength=g.n_lower)
        assert np.all(sup <= (du[u] - 1) * (dl[v] - 1))
        assert np.all(sup <= g.m - 1)
        s1, _, _ = osup(g, orientation=1)
        s2, _, _ = osup(g, orientation=2)
        assert np.array_equal(s1, s2)
        rng = np.random.default_rng(0)
        pick = rng.choice(g.m, size=min(200, g.m), replace=False)
        assert np.array_equal(oracle.edge_support(g.n_upper, g.n_lower, g.row_ptr, g.col, pick), sup[pick])


def test_bitruss_invariants(medium):
    for g in medium:
        sup, bf, _ = osup(g)
        phi, st = ophi(g)
        assert np.all(phi >= 0) and np.all(phi <= sup)
        assert st["destroyed"] == bf
        # max phi is at most k_max: the largest k with at least k edges of support >= k
        s = np.sort(sup)[::-1]
        kmax = int(np.max(np.minimum(s, np.arange(1, s.size + 1)))) if s.size else 0
        assert phi.max() <= kmax
        h, mp = graphs.relabel(g, 1)
        ph, _ = ophi(h)
        assert np.array_equal(ph[mp], phi)
        sh, _, _ = osup(h)
        assert np.array_equal(sh[mp], sup)
        h, mp = graphs.swap_layers(g)
        ph, _ = ophi(h)
        assert np.array_equal(ph[mp], phi)


def test_disjoint_union(medium):
    a, b = medium[1], medium[2]
    pa, _ = ophi(a)
    pb, _ = ophi(b)
    pu, _ = ophi(graphs.disjoint_union(a, b))
    ua, _ = a.edges()
    ub, _ = b.edges()
    # union edges are upper-major: all of a's rows come first
    assert np.array_equal(pu, np.concatenate([pa, pb]))


def test_k_bitruss_fixpoint(medium):
    """{phi >= k} is a subgraph where every edge has >= k butterflies, and no
    edge outside it survives the greatest-fixpoint deletion from G."""
    for g in medium[1:]:
        phi, _ = ophi(g)
        for k in sorted(set(np.unique(phi).tolist()) | {int(phi.max()) + 1}):
            if k == 0:
                continue
            keep = np.ones(g.m, dtype=bool)
            while True:
                h, old = graphs.induced_edges(g, keep)
                s, _, _ = osup(h)
                drop = s < k
                if not drop.any():
                    break
                keep[old[drop]] = False
            assert np.array_equal(keep, phi >= k), k


def test_index_definition_invariants():
    cases = [graphs.random_dense(8, 9, 0.6, s) for s in range(6)]
    cases += [synth.uniform(60, 70, 700, 2)]
    for g in cases:
        sup, bf, _ = osup(g)
        bl = index_def.blooms(g.n_upper, g.n_lower, g.row_ptr, g.col)
        assert sum(math.comb(len(w), 2) for _, _, w in bl) == bf      # Lemmas 1, 3
        acc = np.zeros(g.m, dtype=np.int64)
        for _, _, w in bl:
            seen = [e for pair in w for e in pair]
            assert len(seen) == len(set(seen))                          # Lemma 4
            for e in seen:
                acc[e] += len(w) - 1                                    # Lemma 2
        assert np.array_equal(acc, sup)
        key = index_def.priority_keys(g.n_upper, g.n_lower, g.row_ptr, g.col)
        nbr, _ = index_def._neighbours(g.n_upper, g.n_lower, g.row_ptr, g.col)
        for x in range(g.n_lower + g.n_upper):
            want = [(a, z, w) for a, z, w in bl if a == x]
            got = index_def.blooms_at(x, g.n_upper, g.n_lower, g.row_ptr, g.col, key, nbr)
            assert [(a, z) for a, z, _ in got] == [(a, z) for a, z, _ in want]
            assert [len(ys) for _, _, ys in got] == [len(w) for _, _, w in want]


# --- k-bitruss components (oracle/query.py) ------------------------------------

def _union_of(parts):
    """Disjoint union of graphs given as (n_upper, n_lower, edge list) triples."""
    from paper_2001_06111_amd import synth as _s
    edges, nu, nl = [], 0, 0
    for a, b, es in parts:
        edges += [(u + nu, v + nl) for u, v in es]
        nu += a
        nl += b
    return _s.from_edges(nu, nl, edges)


def test_components_of_disjoint_bicliques_closed_form():
    """K_{3,3} (phi 4 on every edge), K_{2,4} (phi 3), a 5-star (phi 0): H_k has one
    component per part whose closed-form (a-1)(b-1) reaches k."""
    from oracle.query import bitruss_components
    parts = [(3, 3, [(u, v) for u in range(3) for v in range(3)]),
             (2, 4, [(u, v) for u in range(2) for v in range(4)]),
             (1, 5, [(0, v) for v in range(5)])]
    g = _union_of(parts)
    phi = np.array([4] * 9 + [3] * 8 + [0] * 5)
    for k, want in [(0, 3), (1, 2), (3, 2), (4, 1), (5, 0)]:
        comp, c = bitruss_components(g.n_upper, g.n_lower, g.row_ptr, g.col, phi, k)
        assert c == want
        assert np.all((comp >= 0) == (phi >= k))
    comp, c = bitruss_components(g.n_upper, g.n_lower, g.row_ptr, g.col, phi, 1)
    assert list(comp) == [0] * 9 + [1] * 8 + [-1] * 5  # numbered by smallest edge id


def test_components_match_library_routine():
    """On random graphs and thresholds, the partition equals scipy's connected
    components of the edge-induced subgraph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    from oracle.query import bitruss_components
    rng = np.random.default_rng(5)
    for t in range(6):
        g = graphs.random_dense(int(rng.integers(5, 30)), int(rng.integers(5, 30)), 0.15, 40 + t)
        phi = rng.integers(0, 4, size=g.m)
        k = int(rng.integers(0, 4))
        comp, c = bitruss_components(g.n_upper, g.n_lower, g.row_ptr, g.col, phi, k)
        u, v = g.edges()
        sel = phi >= k
        n = g.n_upper + g.n_lower
        a = sp.coo_matrix((np.ones(sel.sum()), (g.n_lower + u[sel], v[sel])), shape=(n, n))
        _, lab = connected_components(a, directed=False)
        ids = np.nonzero(sel)[0]
        # same partition of the selected edges
        pairs = {}
        for e in ids:
            pairs.setdefault(lab[v[e]], set()).add(comp[e])
        assert all(len(x) == 1 for x in pairs.values())
        assert len(pairs) == c and len(set(comp[ids])) == c
        firsts = [int(ids[comp[ids] == i][0]) for i in range(c)]
        assert firsts == sorted(firsts)


def test_components_of_the_worked_example():
    """Section II's example: H_2 (the six edges of bitruss number 2) and H_1 are
    each one connected group."""
    from oracle.query import bitruss_components
    for grey in (True, False):
        g, nm, fx = graphs.worked_example(grey)
        phi = np.zeros(g.m, dtype=np.int64)  # grey edges: 0
        for i in range(9):
            phi[nm[f"e{i}"]] = fx["phi"][f"e{i}"]
        for k in (1, 2):
            _, c = bitruss_components(g.n_upper, g.n_lower, g.row_ptr, g.col, phi, k)
            assert c == 1
