"""The allocator hook, BT_ENOMEM and the serving engine's memory accounting,
through the C ABI on the GPU."""
import re
import threading

import numpy as np
import pytest
import torch

from paper_2001_06111_amd import binding, synth
from tests.gpu_util import oracle_all, upload

pytestmark = pytest.mark.gpu


class Hook:
    """A torch-backed allocator that records request sizes and can refuse
    every request above a size limit."""

    def __init__(self, limit=None):
        self.limit = limit
        self.sizes, self.live = [], {}
        self.frees = 0
        self.errors = []
        self.mu = threading.Lock()

    def alloc(self, n):
        with self.mu:
            self.sizes.append(n)
            if self.limit is not None and n > self.limit:
                return None
        p = torch.cuda.caching_allocator_alloc(n)
        with self.mu:
            self.live[p] = n
        return p

    def free(self, p, n):
        with self.mu:
            if self.live.pop(p, None) != n:
                self.errors.append((p, n))
            self.frees += 1
        torch.cuda.caching_allocator_delete(p)

    def install(self):
        binding.bt_set_allocator(self.alloc, self.free)


@pytest.fixture(autouse=True)
def _default_allocator():
    binding.bt_release_workspace()
    yield
    binding.bt_release_workspace()
    binding.bt_set_allocator()


def test_injected_failure_returns_enomem_then_recovers():
    g = synth.scaled_chunglu(40_000, seed=11)
    dg = upload(g)
    rec = Hook()
    rec.install()
    binding.bt_decompose(dg)
    torch.cuda.synchronize()
    binding.bt_release_workspace()
    assert rec.frees == len(rec.sizes) and not rec.live and not rec.errors  # all returned
    big = max(rec.sizes)
    fail = Hook(limit=big - 1)
    fail.install()
    with pytest.raises(binding.BtError) as ei:
        binding.bt_decompose(dg)
    assert ei.value.status == binding.BT_ENOMEM
    sizes = [int(s) for s in re.findall(r"allocation of (\d+) bytes", str(ei.value))]
    assert sizes and sizes[0] > big - 1
    # The library is usable afterwards: first through a working hook, then
    # through hipMalloc again.
    ok = Hook()
    ok.install()
    sup, phi, _ = binding.bt_decompose(dg)
    osup, _, ophi = oracle_all(g)
    assert np.array_equal(sup.cpu().numpy(), osup) and np.array_equal(phi.cpu().numpy(), ophi)
    binding.bt_set_allocator()
    binding.bt_release_workspace()
    assert not ok.live and not fail.live
    sup2, phi2, _ = binding.bt_decompose(dg)
    assert torch.equal(phi2, phi) and torch.equal(sup2, sup)


def test_torch_caching_allocator_owns_the_workspace():
    g = synth.scaled_chunglu(30_000, seed=12)
    dg = upload(g)
    before = torch.cuda.memory_allocated()
    binding.use_torch_allocator()
    sup, phi, _ = binding.bt_decompose(dg)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before
    assert held > 0  # the workspace now lives in torch's pool
    osup, _, ophi = oracle_all(g)
    assert np.array_equal(phi.cpu().numpy(), ophi)
    binding.bt_release_workspace()
    assert torch.cuda.memory_allocated() - before < held


def _engine_run(gs, hook, slots=1, budget=0):
    hook.install()
    eng = binding.BtEngine(hbm_budget=budget, slots=slots)
    dgs = [upload(g) for g in gs]
    for i, d in enumerate(dgs):
        eng.bt_engine_submit(d, i)
    eng.bt_engine_drain()
    done = dict(eng.bt_engine_poll())
    mem = eng.bt_engine_memory()
    eng.bt_engine_destroy()
    binding.bt_set_allocator()
    torch.cuda.synchronize()
    return eng.results, done, mem


def test_engine_enomem_fails_only_that_request():
    small = [synth.batch_graph(i) for i in (0, 1, 2, 5)]
    small = [g for g in small if g.m < (1 << 14)][:3]
    big = synth.scaled_chunglu(120_000, seed=13)  # another size class: its own batch
    assert len(small) == 3 and big.m >= (1 << 14)
    rec_small, rec_big = Hook(), Hook()
    _engine_run(small, rec_small)
    _engine_run([big], rec_big)
    limit = max(rec_small.sizes)
    assert max(rec_big.sizes) > limit
    assert big.n_lower * 4 + 256 < limit  # its submit-time estimate still allocates
    res, done, _ = _engine_run(small + [big], Hook(limit=limit))
    assert done[len(small)] == binding.BT_ENOMEM
    for i, g in enumerate(small):
        assert done[i] == binding.BT_OK
        _, _, ophi = oracle_all(g)
        assert np.array_equal(res[i][2].cpu().numpy(), ophi)


def test_engine_two_slots_stay_within_budget():
    """With a budget that holds about one large request, two slots share it:
    the sum of what the slots hold plus what their running batches may add
    never exceeds the budget, and results do not change."""
    gs = [synth.batch_graph(i) for i in range(40)] + [synth.scaled_chunglu(60_000, seed=14),
                                                       synth.scaled_chunglu(70_000, seed=15)]
    alone = max(_engine_run([g], Hook())[2]["peak_committed"] for g in gs)
    res0, done0, mem0 = _engine_run(gs, Hook(), slots=2)
    assert all(s == binding.BT_OK for s in done0.values())
    budget = alone * 5 // 4
    res, done, mem = _engine_run(gs, Hook(), slots=2, budget=budget)
    assert all(s == binding.BT_OK for s in done.values()), done
    assert mem["budget"] == budget
    assert mem["peak_committed"] <= budget and mem["peak_held"] <= budget, mem
    for i in range(len(gs)):
        assert torch.equal(res[i][2], res0[i][2])


def test_engine_request_mix_alone_equals_mix():
    """The serving mix (pool graphs with 2M-edge request graphs, arriving
    while others run, two slots): every result equals the plain
    single-graph decomposition of the same request, and request graph 0
    equals the oracle's digest."""
    import hashlib
    import json
    import os
    import time
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json")))
    small = [synth.batch_graph(i) for i in range(30)]
    big = [synth.big_serving_graph(0), synth.big_serving_graph(1)]
    gs = small[:10] + big[:1] + small[10:20] + big[1:] + small[20:]
    dgs = [upload(g) for g in gs]
    eng = binding.BtEngine(slots=2)
    for i, d in enumerate(dgs):
        eng.bt_engine_submit(d, i)
        time.sleep(0.005)
    eng.bt_engine_drain()
    done = dict(eng.bt_engine_poll())
    eng.bt_engine_destroy()
    assert sorted(done) == list(range(len(gs)))
    for i, d in enumerate(dgs):
        assert done[i] == binding.BT_OK
        _, phi, _ = binding.bt_decompose(d, want_sup=False)
        assert torch.equal(eng.results[i][2], phi), gs[i].name
    i0 = gs.index(big[0])
    want = gold["big:1"]["per_graph"][0]["phi_sha256"]
    got = hashlib.sha256(eng.results[i0][2].cpu().numpy().astype("<i8").tobytes()).hexdigest()
    assert got == want


def test_caller_driven_engine_steps():
    """An engine created with slots = -1 has no worker threads: each
    bt_engine_step admits one batch as a free slot would and decomposes it
    on this thread; every result equals the plain decomposition; drain
    steps until the queue is empty; a threaded engine refuses steps."""
    gs = [synth.batch_graph(i) for i in range(24)] + [synth.scaled_chunglu(60_000, seed=16)]
    dgs = [upload(g) for g in gs]
    eng = binding.BtEngine(slots=-1)
    try:
        assert eng.bt_engine_step() == 0  # nothing queued
        for i, d in enumerate(dgs):
            eng.bt_engine_submit(d, i)
        n1 = eng.bt_engine_step()
        first = dict(eng.bt_engine_poll())
        assert n1 > 0 and len(first) == n1
        steps, total = 1, n1
        while True:
            k = eng.bt_engine_step()
            if k == 0:
                break
            steps += 1
            total += k
        done = dict(first)
        done.update(eng.bt_engine_poll())
        assert total == len(gs) and sorted(done) == list(range(len(gs)))
        assert all(st == binding.BT_OK for st in done.values())
        st = eng.bt_engine_stats()
        assert st["batches"] == steps >= 2 and st["queued"] == 0  # two size classes at least
        for i, d in enumerate(dgs):
            _, phi, _ = binding.bt_decompose(d, want_sup=False)
            assert torch.equal(eng.results[i][2], phi), gs[i].name
        for i, d in enumerate(dgs[:5]):
            eng.bt_engine_submit(d, 100 + i)
        eng.bt_engine_drain()
        assert sorted(dict(eng.bt_engine_poll())) == [100, 101, 102, 103, 104]
    finally:
        eng.bt_engine_destroy()
    threaded = binding.BtEngine(slots=1)
    try:
        with pytest.raises(binding.BtError) as ei:
            threaded.bt_engine_step()
        assert ei.value.status == binding.BT_EINVAL
    finally:
        threaded.bt_engine_destroy()
