"""Full-size parity: the 5M-edge Chung-Lu workload and 512 pool graphs against the oracle.

Bitruss numbers and supports are compared bit for bit through SHA-256
digests of the oracle's outputs (tests/golden/digests.json, written by
make_digests.py from the oracle); supports of sampled edges are also
recounted one by one from the definition.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2001_06111_amd import binding, synth

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json")))


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def c1():
    g = synth.plain_chunglu_5m()
    sup, phi, st = binding.bt_decompose(binding.DeviceGraph.upload(g), stats=True)
    torch.cuda.synchronize()
    return g, sup.cpu().numpy(), phi.cpu().numpy(), st


def test_chunglu5m_digests(c1):
    g, sup, phi, st = c1
    want = GOLD[g.name]
    assert want["generator_version"] == synth.GENERATOR_VERSION
    assert st["butterflies"] == want["butterflies"]
    assert sha(sup) == want["sup_sha256"]
    assert sha(phi) == want["phi_sha256"]
    assert st["levels"] == want["levels"] and st["max_phi"] == want["max_phi"]


def test_chunglu5m_sampled_supports_and_invariants(c1):
    g, sup, phi, st = c1
    rng = np.random.default_rng(0)
    pick = rng.choice(g.m, size=300, replace=False)
    assert np.array_equal(oracle.edge_support(g.n_upper, g.n_lower, g.row_ptr, g.col, pick), sup[pick])
    assert sup.sum() == 4 * st["butterflies"]
    assert np.all(phi >= 0) and np.all(phi <= sup)


def test_uniform10k_digests():
    g = synth.plain_uniform_10k()
    sup, phi, st = binding.bt_decompose(binding.DeviceGraph.upload(g), stats=True)
    want = GOLD[g.name]
    assert sha(sup.cpu().numpy()) == want["sup_sha256"] and sha(phi.cpu().numpy()) == want["phi_sha256"]


def test_pool512_batched_digests():
    """The first 512 graphs of the many-small-graphs pool, decomposed as one
    batched call (each graph at its own level): the concatenated supports and
    bitruss numbers equal the oracle's, bit for bit."""
    want = GOLD["pool:512"]
    assert want["generator_version"] == synth.GENERATOR_VERSION
    gs = [synth.batch_graph(i) for i in range(512)]
    dgs = [binding.DeviceGraph.upload(g) for g in gs]
    sups, phis, st = binding.bt_decompose_batch(dgs, stats=True)
    torch.cuda.synchronize()
    hs, hp = hashlib.sha256(), hashlib.sha256()
    for s, p in zip(sups, phis):
        hs.update(np.ascontiguousarray(s.cpu().numpy(), dtype="<i8").tobytes())
        hp.update(np.ascontiguousarray(p.cpu().numpy(), dtype="<i8").tobytes())
    assert st["butterflies"] == want["butterflies"]
    assert hs.hexdigest() == want["sup_sha256"]
    assert hp.hexdigest() == want["phi_sha256"]
    for i, g in enumerate(want["per_graph"]):
        assert sha(phis[i].cpu().numpy()) == g["phi_sha256"]


def test_request_graph_2m_digest():
    """The first 2M-edge graph of the request stream (the serving workload's
    large class), decomposed alone and through the serving engine: supports
    and bitruss numbers equal the oracle's, bit for bit."""
    want = GOLD["big:1"]
    assert want["generator_version"] == synth.GENERATOR_VERSION
    g = synth.big_serving_graph(0)
    dg = binding.DeviceGraph.upload(g)
    sup, phi, st = binding.bt_decompose(dg, stats=True)
    assert st["butterflies"] == want["butterflies"]
    assert sha(sup.cpu().numpy()) == want["sup_sha256"]
    assert sha(phi.cpu().numpy()) == want["phi_sha256"]
    eng = binding.BtEngine()
    try:
        eng.bt_engine_submit(dg, 7)
        eng.bt_engine_drain()
        assert eng.bt_engine_poll() == [(7, binding.BT_OK)]
        status, _, phi_e = eng.results[7]
        assert sha(phi_e.cpu().numpy()) == want["phi_sha256"]
    finally:
        eng.bt_engine_destroy()


def test_request_graphs_digests():
    """Every 2M-edge request graph with an oracle digest, decomposed four at
    a time as one union (the serving engine's large-class batch, one shared
    level): supports, totals and bitruss numbers equal the oracle's."""
    path = os.path.join(os.path.dirname(__file__), "golden", "digests_requests.json")
    per = json.load(open(path))["per_graph"] if os.path.exists(path) else {}
    js = sorted(int(j) for j in per)
    if not js:
        pytest.skip("no request-graph digests beyond graph 0")
    for k in range(0, len(js), 4):
        part = js[k:k + 4]
        dgs = [binding.DeviceGraph.upload(synth.big_serving_graph(j)) for j in part]
        sups, phis, _ = binding.bt_decompose_batch(dgs)
        for j, sup, phi in zip(part, sups, phis):
            want = per[str(j)]
            assert want["generator_version"] == synth.GENERATOR_VERSION
            assert int(sup.sum().item()) == 4 * want["butterflies"], j
            assert sha(sup.cpu().numpy()) == want["sup_sha256"], j
            assert sha(phi.cpu().numpy()) == want["phi_sha256"], j
        del dgs, sups, phis


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_pool4096_batched_digests():
    """The whole 4,096-graph pool as one batched call (as the benchmark times
    it): the concatenated supports and bitruss numbers equal the oracle's."""
    import concurrent.futures as cf
    want = GOLD["pool:4096"]
    assert want["generator_version"] == synth.GENERATOR_VERSION
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        gs = list(ex.map(synth.batch_graph, range(4096), chunksize=32))
    dgs = [binding.DeviceGraph.upload(g) for g in gs]
    sups, phis, st = binding.bt_decompose_batch(dgs, stats=True)
    torch.cuda.synchronize()
    hs, hp = hashlib.sha256(), hashlib.sha256()
    for s, p in zip(sups, phis):
        hs.update(np.ascontiguousarray(s.cpu().numpy(), dtype="<i8").tobytes())
        hp.update(np.ascontiguousarray(p.cpu().numpy(), dtype="<i8").tobytes())
    assert st["butterflies"] == want["butterflies"]
    assert hs.hexdigest() == want["sup_sha256"]
    assert hp.hexdigest() == want["phi_sha256"]


def test_pc_fullsize_digests(c1):
    """BiT-PC (the progressive compression of Section V-C) at full size: on
    the 5M-edge graph and on the 2M-edge request graph its bitruss numbers
    equal the oracle's, bit for bit."""
    g, _, _, _ = c1
    _, phi, st = binding.bt_decompose_pc(binding.DeviceGraph.upload(g), tau=0.05, stats=True,
                                         want_sup=False)
    assert sha(phi.cpu().numpy()) == GOLD[g.name]["phi_sha256"]
    assert st["passes"] > 1
    b = synth.big_serving_graph(0)
    _, phi, _ = binding.bt_decompose_pc(binding.DeviceGraph.upload(b), tau=0.1, want_sup=False)
    assert sha(phi.cpu().numpy()) == GOLD["big:1"]["phi_sha256"]


@pytest.mark.slow
def test_components_fullsize(c1):
    """Connected components of two top k-bitrusses of the 5M-edge graph (the
    bitruss numbers are the oracle's, by the digest test) against the
    oracle's breadth-first search."""
    from oracle import query
    g, _, phi, _ = c1
    dg = binding.DeviceGraph.upload(g)
    dphi = torch.from_numpy(phi).cuda()
    for k in (int(np.percentile(phi, 99.9)), int(phi.max())):
        comp, n = binding.bt_bitruss_components(dg, dphi, k)
        want, wn = query.bitruss_components(g.n_upper, g.n_lower, g.row_ptr, g.col, phi, k)
        assert n == wn and np.array_equal(comp.cpu().numpy(), want), k
