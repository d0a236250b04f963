"""The seeded input generators, on the CPU: valid CSRs of the stated shapes,
reproducible from their seeds, and the stream and sample recipes as stated."""
import numpy as np
import pytest

from paper_2001_06111_amd import synth


def assert_valid_csr(g):
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.m == g.col.size
    assert np.all(np.diff(g.row_ptr) >= 0)
    assert g.col.dtype == np.int32
    if g.m:
        assert g.col.min() >= 0 and g.col.max() < g.n_lower
    for x in range(g.n_upper):
        row = g.col[g.row_ptr[x]:g.row_ptr[x + 1]]
        assert np.all(np.diff(row) > 0), x  # strictly increasing: no duplicate edges


def same(a, b):
    return (a.n_upper, a.n_lower, a.m) == (b.n_upper, b.n_lower, b.m) and \
        np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)


def test_uniform_shape_and_seed():
    g = synth.uniform(100, 150, 1000, 5)
    assert (g.n_upper, g.n_lower, g.m) == (100, 150, 1000)
    assert_valid_csr(g)
    assert same(g, synth.uniform(100, 150, 1000, 5))
    assert not same(g, synth.uniform(100, 150, 1000, 6))


def test_expected_degrees_sum_cap_and_order():
    d = synth.expected_degrees(1000, 20_000, 2.1, 200.0)
    assert d.sum() == pytest.approx(20_000)
    assert d.max() <= 200.0 + 1e-9
    assert np.all(np.diff(d) <= 1e-9)  # non-increasing before the permutation
    with pytest.raises(ValueError):
        synth.expected_degrees(10, 1000, 2.1, 50.0)  # cap * n < m


def test_chung_lu_shape_and_seed():
    g = synth.chung_lu(300, 500, 4000, 2.1, 2.5, 200.0, 200.0, 9)
    assert (g.n_upper, g.n_lower, g.m) == (300, 500, 4000)
    assert_valid_csr(g)
    assert same(g, synth.chung_lu(300, 500, 4000, 2.1, 2.5, 200.0, 200.0, 9))
    # ids independent of degree: the highest-degree vertex is not always id 0
    du = np.diff(g.row_ptr)
    assert int(np.argmax(du)) != 0 or int(np.argmax(np.bincount(g.col))) != 0
    with pytest.raises(ValueError):
        synth.chung_lu(3, 3, 10, 2.1, 2.1, 3.0, 3.0, 0)


def test_scaled_chunglu_keeps_edge_count():
    g = synth.scaled_chunglu(20_000, seed=4)
    assert g.m == 20_000
    assert_valid_csr(g)


@pytest.mark.parametrize("i", [0, 1, 7, 123, 4095])
def test_batch_graph_recipe(i):
    g = synth.batch_graph(i)
    assert 50 <= g.n_upper <= 20000 and 50 <= g.n_lower <= 20000
    assert g.m <= 200_000 and g.m <= (g.n_upper * g.n_lower) // 4
    assert g.m >= min(200, (g.n_upper * g.n_lower) // 4)
    assert_valid_csr(g)
    assert same(g, synth.batch_graph(i))


def test_serving_arrivals_recipe():
    a = synth.serving_arrivals(duration=5.0)
    t = np.array([x[0] for x in a])
    assert np.all(np.diff(t) > 0) and t[0] > 0 and t[-1] <= 5.0
    assert 850 <= len(a) <= 1150  # Poisson, 200/s for 5 s
    kinds = [x[1] for x in a]
    big = sum(k == "big" for k in kinds)
    assert set(kinds) <= {"small", "big"} and 0.02 < big / len(a) < 0.09
    assert all(0 <= x[2] < (4096 if x[1] == "small" else 32) for x in a)
    assert a == synth.serving_arrivals(duration=5.0)
    assert a[:10] == synth.serving_arrivals(duration=60.0)[:10]  # a window is a prefix


def test_vertex_sample_is_an_induced_subgraph():
    g = synth.chung_lu(200, 300, 3000, 2.1, 2.1, 150.0, 150.0, 3)
    s = synth.vertex_sample(g, 0.5, 2027)
    assert (s.n_upper, s.n_lower) == (100, 150)
    assert_valid_csr(s)
    rng = np.random.default_rng(2027)
    keep_u = np.sort(rng.permutation(g.n_upper)[:100])
    keep_l = np.sort(rng.permutation(g.n_lower)[:150])
    u, v = g.edges()
    inside = np.isin(u, keep_u) & np.isin(v, keep_l)
    assert s.m == int(inside.sum())
    su, sv = s.edges()
    assert np.array_equal(np.sort(keep_u[su] * g.n_lower + keep_l[sv]),
                          np.sort(u[inside] * g.n_lower + v[inside]))
