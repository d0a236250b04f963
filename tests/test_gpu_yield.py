"""The persistent peel giving the device to a smaller peel and resuming.

A launch that stops after a rebuild of its active set and is launched again
must give exactly the decomposition of an uninterrupted peel, with the same
rounds, levels and updates; in the serving engine a small batch that comes
while a large request peels runs in between, and every result equals the
one computed alone."""
import hashlib
import json
import os
import time

import numpy as np
import pytest
import torch

from paper_2001_06111_amd import binding, synth
from tests.gpu_util import oracle_all, upload

pytestmark = pytest.mark.gpu

SAME = ("rounds", "levels", "support_updates", "bloom_visits", "wedge_visits", "max_phi",
        "support_updates_unbatched")


@pytest.mark.parametrize("m,seed", [(120_000, 21), (400_000, 22)])
def test_forced_yield_resumes_exactly(monkeypatch, m, seed):
    g = synth.scaled_chunglu(m, seed=seed)
    dg = upload(g)
    sup0, phi0, st0 = binding.bt_decompose(dg, stats=True)
    monkeypatch.setenv("BT_PEEL_YIELD", "1")
    sup1, phi1, st1 = binding.bt_decompose(dg, stats=True)
    monkeypatch.delenv("BT_PEEL_YIELD")
    assert st0["peel_yields"] == 0 and st0["peel_launches"] == 1
    assert st1["peel_yields"] >= 1, st1
    assert st1["peel_launches"] == st1["peel_yields"] + 1
    for k in SAME:
        assert st1[k] == st0[k], k
    assert torch.equal(sup0, sup1) and torch.equal(phi0, phi1)
    if m <= 120_000:
        osup, _, ophi = oracle_all(g)
        assert np.array_equal(sup1.cpu().numpy(), osup)
        assert np.array_equal(phi1.cpu().numpy(), ophi)


def test_forced_yield_in_progressive_passes(monkeypatch):
    """BiT-PC's passes fix part of the edges and start at a minimum level; a
    resumed launch keeps both."""
    g = synth.scaled_chunglu(150_000, seed=23)
    dg = upload(g)
    _, phi0, _ = binding.bt_decompose(dg, want_sup=False)
    monkeypatch.setenv("BT_PEEL_YIELD", "1")
    _, phi1, st1 = binding.bt_decompose_pc(dg, tau=0.3, want_sup=False, stats=True)
    monkeypatch.delenv("BT_PEEL_YIELD")
    assert st1["peel_yields"] >= 1 and st1["passes"] > 1
    assert torch.equal(phi0, phi1)


def test_forced_yield_in_batch_peel(monkeypatch):
    """The batch peel (each graph at its own level) resumes at the round
    where it stopped: same numbers and the same rounds."""
    gs = [synth.batch_graph(i) for i in range(40)]
    dgs = [upload(g) for g in gs]
    sups0, phis0, st0 = binding.bt_decompose_batch(dgs, stats=True)
    monkeypatch.setenv("BT_PEEL_YIELD", "1")
    sups1, phis1, st1 = binding.bt_decompose_batch(dgs, stats=True)
    monkeypatch.delenv("BT_PEEL_YIELD")
    assert st0["peel_yields"] == 0
    assert st1["peel_yields"] >= 1 and st1["peel_launches"] == st0["peel_launches"] + st1["peel_yields"]
    for k in ("rounds", "levels", "support_updates", "bloom_visits", "wedge_visits", "max_phi"):
        assert st1[k] == st0[k], k
    for i, g in enumerate(gs):
        assert torch.equal(phis0[i], phis1[i]) and torch.equal(sups0[i], sups1[i]), g.name
    for i in (0, 1, 2):
        osup, _, ophi = oracle_all(gs[i])
        assert np.array_equal(phis1[i].cpu().numpy(), ophi)


def test_engine_small_batches_run_while_a_large_request_peels():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json")))
    big = synth.big_serving_graph(0)
    small = [g for g in (synth.batch_graph(i) for i in range(48)) if g.m < (1 << 14)][:12]
    db = upload(big)
    ds = [upload(g) for g in small]
    alone = [binding.bt_decompose(d, want_sup=False)[1] for d in ds]
    eng = binding.BtEngine(slots=2)
    eng.bt_engine_submit(db, 0)
    order, sent = [], {}
    nid = 1
    t_end = time.perf_counter() + 60
    # Offer a small request every 20 ms until the large one is done.
    while 0 not in order and time.perf_counter() < t_end:
        sent[nid] = nid % len(ds)
        eng.bt_engine_submit(ds[sent[nid]], nid)
        nid += 1
        time.sleep(0.02)
        order += [rid for rid, _ in eng.bt_engine_poll()]
    eng.bt_engine_drain()
    order += [rid for rid, _ in eng.bt_engine_poll()]
    st = eng.bt_engine_stats()
    eng.bt_engine_destroy()
    assert 0 in order and sorted(order) == list(range(nid))
    assert all(eng.results[i][0] == binding.BT_OK for i in order)
    # Some small request finished while the large one was still running,
    # and the large peel gave way at least once.
    assert order.index(0) > 0
    assert st["peel_yields"] >= 1, st
    for rid, k in sent.items():
        assert torch.equal(eng.results[rid][2], alone[k]), (rid, small[k].name)
    want = gold["big:1"]["per_graph"][0]["phi_sha256"]
    got = hashlib.sha256(eng.results[0][2].cpu().numpy().astype("<i8").tobytes()).hexdigest()
    assert got == want
