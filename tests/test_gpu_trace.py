"""The peel round by round on the paper's running example (bt_decompose_trace).

Section V-B's example of the batch peel: the first round (minimum support 1)
removes e6, e7, e8 together, which lowers e5 from 3 to 2 and leaves bloom B1
(dominant vertices v1, v2; other vertices u2, u3) with no butterfly; the
second round removes e0..e5 together and empties bloom B0.  The RemoveEdge
example of Section IV-A: e6's removal costs e5 exactly one butterfly (its
twin in B1 loses k - 1 = 1), so e5 ends round 1 at 3 - (2 - 1) = 2.
"""
import numpy as np
import pytest

from paper_2001_06111_amd import binding
from tests import graphs
from tests.gpu_util import oracle_all, upload

pytestmark = pytest.mark.gpu


def bf(k):
    """Butterflies of a bloom with k live wedges (Lemma 8)."""
    return k * (k - 1) // 2


def _bloom_of(tr, edges):
    """Wedges both of whose edges lie in `edges`."""
    ea, eb = tr["wedge_ea"], tr["wedge_eb"]
    return [w for w in range(len(ea)) if ea[w] in edges and eb[w] in edges]


def test_trace_running_example_9edge():
    g, nm, fx = graphs.worked_example(False)
    tr = binding.bt_decompose_trace(upload(g))
    e = [nm[f"e{i}"] for i in range(9)]
    assert tr["level"].tolist() == [1, 2]
    assert sorted(np.nonzero(tr["removed"][0])[0].tolist()) == sorted(e[6:9])
    assert sorted(np.nonzero(tr["removed"][1])[0].tolist()) == sorted(e[0:6])
    assert tr["sup"][0][e[5]] == fx["support_e5_after_removing_e6"] == 2
    b1 = _bloom_of(tr, {e[5], e[6], e[7], e[8]})
    b0 = _bloom_of(tr, set(e[0:6]))
    assert len(b1) == 2 and len(b0) == 3
    k1, k0 = tr["wedge_k"][:, b1], tr["wedge_k"][:, b0]
    assert np.all(bf(k1[0]) == 0)                       # B1 emptied by round 1
    assert np.all(bf(k0[0]) == fx["bloom_B0_butterflies"])  # B0 untouched
    assert np.all(bf(k0[1]) == 0)                       # B0 emptied by round 2
    _, _, ophi = oracle_all(g)
    assert np.array_equal(tr["phi"].cpu().numpy(), ophi)


def test_trace_running_example_11edge():
    g, nm, fx = graphs.worked_example(True)
    tr = binding.bt_decompose_trace(upload(g))
    e = [nm[f"e{i}"] for i in range(9)]
    grey = {nm["grey0"], nm["grey1"]}
    assert tr["level"].tolist() == [0, 1, 2]
    assert set(np.nonzero(tr["removed"][0])[0].tolist()) == grey
    assert sorted(np.nonzero(tr["removed"][1])[0].tolist()) == sorted(e[6:9])
    assert sorted(np.nonzero(tr["removed"][2])[0].tolist()) == sorted(e[0:6])
    assert tr["sup"][1][e[5]] == 2
    # every edge is removed exactly once, at its bitruss number
    assert np.all(tr["removed"].sum(axis=0) == 1)
    phi = tr["phi"].cpu().numpy()
    for k, lv in enumerate(tr["level"]):
        assert np.all(phi[tr["removed"][k]] == lv)


def test_trace_limits():
    g, _, _ = graphs.worked_example(True)
    with pytest.raises(binding.BtError) as ei:
        binding.bt_decompose_trace(upload(g), max_rounds=2)
    assert ei.value.status == binding.BT_EOVERFLOW
