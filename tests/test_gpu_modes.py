"""The peel's alternative launch forms give the oracle's results.

Besides the persistent cooperative kernel the peel can run as two kernels
per round, replayed from captured HIP graphs (BT_PEEL_MODE=graph) or
launched directly (BT_PEEL_GRAPH=0), with the active set rebuilt by the
host; batches can use the shared-level peel over their union
(BT_BATCH_PEEL=union) instead of per-graph levels.  Each captured graph is
replayed many times per decomposition, with host work and synchronisation
between replays, and again by a second decomposition that reuses it.
"""
import numpy as np
import pytest

from paper_2001_06111_amd import binding, synth
from tests import graphs
from tests.gpu_util import oracle_all, upload

pytestmark = pytest.mark.gpu


def _cases():
    return [graphs.worked_example(True)[0], graphs.k2_1001(), synth.complete(7, 9),
            synth.scaled_chunglu(20_000, seed=3), synth.plain_uniform_10k(),
            graphs.random_dense(30, 25, 0.6, 1)]


@pytest.mark.parametrize("replay", ["1", "0"])
def test_round_kernels(monkeypatch, replay):
    monkeypatch.setenv("BT_PEEL_MODE", "graph")
    monkeypatch.setenv("BT_PEEL_GRAPH", replay)
    for g in _cases():
        osup, obf, ophi = oracle_all(g)
        dg = upload(g)
        for _ in range(2):
            sup, phi, st = binding.bt_decompose(dg, stats=True)
            assert np.array_equal(sup.cpu().numpy(), osup), g.name
            assert np.array_equal(phi.cpu().numpy(), ophi), g.name
            assert st["butterflies"] == obf
        _, phi_pc, _ = binding.bt_decompose_pc(dg, tau=0.2)
        assert np.array_equal(phi_pc.cpu().numpy(), ophi), g.name


def test_round_kernels_match_persistent_counters(monkeypatch):
    g = synth.scaled_chunglu(200_000, seed=3)
    dg = upload(g)
    _, phi_p, st_p = binding.bt_decompose(dg, stats=True)
    monkeypatch.setenv("BT_PEEL_MODE", "graph")
    _, phi_g, st_g = binding.bt_decompose(dg, stats=True)
    assert np.array_equal(phi_p.cpu().numpy(), phi_g.cpu().numpy())
    for k in ("levels", "max_phi", "support_updates", "bloom_visits"):
        assert st_p[k] == st_g[k], k


def test_batch_union_peel(monkeypatch):
    gs = [synth.batch_graph(i) for i in range(16)]
    dgs = [upload(g) for g in gs]
    monkeypatch.setenv("BT_BATCH_PEEL", "union")
    _, phis, _ = binding.bt_decompose_batch(dgs, stats=True)
    for g, ph in zip(gs, phis):
        assert np.array_equal(ph.cpu().numpy(), oracle_all(g)[2]), g.name
