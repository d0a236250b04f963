"""Checks on the 20M-edge hub-skewed Chung-Lu workload.

Bitruss numbers of vertex-sampled induced subgraphs are compared bit for bit
with the oracle's digests, by the plain peel and by BiT-PC; on the full
graph the two must agree, match the oracle's digest where it has been
written (its peel takes hours here), and satisfy properties that hold at
any size, each computed by the oracle from the GPU's answer:
  * supports: SHA-256 of the oracle's full support vector and the butterfly
    total (tests/golden/digests.json, written by make_digests.py);
  * 0 <= phi_e <= support_e (Lemma 10's bound), and max phi <= k_max, the
    largest k with at least k edges of support >= k (the first threshold of
    BiT-PC, Section V-C: a k-bitruss holds at least k edges of support >= k);
  * soundness: for sampled k, every edge of H_k = {phi >= k} lies in at least
    k butterflies of H_k (Definition 4), recounted by the oracle on H_k;
  * maximality for the top levels: the greatest subgraph of H_{k-1} in which
    every edge has support >= k, found by the oracle's repeated recount,
    is exactly H_k (so no edge of phi = k - 1 belongs to a k-bitruss).
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2001_06111_amd import binding, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(1200)]

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json")))


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def sub_support(g, ids):
    """Oracle supports of the edge-induced subgraph on `ids` (sorted edge ids)."""
    u = np.repeat(np.arange(g.n_upper, dtype=np.int64), np.diff(g.row_ptr))[ids]
    row_ptr = np.zeros(g.n_upper + 1, dtype=np.int64)
    np.add.at(row_ptr, u + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    sup, _, _ = oracle.support(g.n_upper, g.n_lower, row_ptr, g.col[ids])
    return sup


@pytest.fixture(scope="module")
def hub():
    g = synth.plain_hub_20m()
    print(f"[hub20m] generated m={g.m}", flush=True)
    return g


@pytest.fixture(scope="module")
def c2(hub):
    """The plain peel (Algorithm 5) and BiT-PC (Algorithm 7) on the full graph."""
    g = hub
    dg = binding.DeviceGraph.upload(g)
    print("[hub20m] decomposing on the GPU (plain peel)", flush=True)
    sup, phi, st = binding.bt_decompose(dg, stats=True)
    torch.cuda.synchronize()
    print(f"[hub20m] plain: rounds {st['rounds']}, max phi {st['max_phi']}; now BiT-PC", flush=True)
    _, phi_pc, st_pc = binding.bt_decompose_pc(dg, tau=0.05, want_sup=False, stats=True)
    torch.cuda.synchronize()
    print(f"[hub20m] BiT-PC: passes {st_pc['passes']}", flush=True)
    return g, sup.cpu().numpy(), phi.cpu().numpy(), st, phi_pc.cpu().numpy()


def test_hub20m_plain_equals_pc(c2):
    g, sup, phi, st, phi_pc = c2
    assert np.array_equal(phi, phi_pc)


def test_hub20m_phi_digest(c2):
    """Bit-exact against the oracle's full bitruss numbers, once that run
    (hours on a CPU) has written its digest."""
    g, sup, phi, st, phi_pc = c2
    want = GOLD[g.name].get("phi_sha256")
    if want is None:
        pytest.skip("no oracle phi digest for the full 20M-edge graph in digests.json")
    assert sha(phi) == want and sha(phi_pc) == want


SAMPLES = sorted(k for k, v in GOLD.items()
                 if isinstance(v, dict) and v.get("sample", {}).get("of") == "chunglu-100kx2M-m20M-hub")


@pytest.mark.parametrize("key", SAMPLES)
def test_hub20m_vertex_sample_digests(hub, key):
    """Vertex-sampled induced subgraphs of the hub graph (the paper's
    scalability sampling), bit-exact against the oracle by the plain peel
    and by BiT-PC."""
    want = GOLD[key]
    smp = synth.vertex_sample(hub, want["sample"]["fraction"], want["sample"]["seed"])
    assert smp.name == key and smp.m == want["m"]
    dg = binding.DeviceGraph.upload(smp)
    sup, phi, st = binding.bt_decompose(dg, stats=True)
    _, phi_pc, _ = binding.bt_decompose_pc(dg, tau=0.05, want_sup=False)
    torch.cuda.synchronize()
    print(f"[hub20m] {key}: rounds {st['rounds']}", flush=True)
    assert st["butterflies"] == want["butterflies"]
    assert sha(sup.cpu().numpy()) == want["sup_sha256"]
    assert sha(phi.cpu().numpy()) == want["phi_sha256"]
    assert sha(phi_pc.cpu().numpy()) == want["phi_sha256"]


def test_hub20m_supports(c2):
    g, sup, phi, st, _ = c2
    want = GOLD[g.name]
    assert want["generator_version"] == synth.GENERATOR_VERSION
    assert st["butterflies"] == want["butterflies"]
    assert sha(sup) == want["sup_sha256"]


def test_hub20m_phi_bounds(c2):
    g, sup, phi, st, _ = c2
    assert np.all(phi >= 0) and np.all(phi <= sup)
    s = np.sort(sup)[::-1]
    kmax = int(np.max(np.minimum(s, np.arange(1, len(s) + 1))))
    assert int(phi.max()) == st["max_phi"] <= kmax


def test_hub20m_soundness(c2):
    g, sup, phi, st, _ = c2
    pos = np.sort(phi[phi > 0])
    ks = sorted({1, int(pos[len(pos) // 2]), int(pos[int(len(pos) * 0.9)]),
                 int(pos[int(len(pos) * 0.99)]), int(phi.max())})
    for k in ks:
        ids = np.nonzero(phi >= k)[0]
        s = sub_support(g, ids)
        print(f"[hub20m] soundness k={k}: |H_k|={len(ids)}, min support {int(s.min())}", flush=True)
        assert s.min() >= k


def test_hub20m_maximality_top_levels(c2):
    g, sup, phi, st, _ = c2
    levels = np.unique(phi)[::-1][:3]
    for k in levels:
        k = int(k)
        ids = np.nonzero(phi >= k - 1)[0]
        while True:
            s = sub_support(g, ids)
            keep = s >= k
            if keep.all():
                break
            ids = ids[keep]
        print(f"[hub20m] maximality k={k}: fixpoint {len(ids)} edges", flush=True)
        assert np.array_equal(ids, np.nonzero(phi >= k)[0])
