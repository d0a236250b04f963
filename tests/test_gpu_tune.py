"""Launch parameters never change a result; the autotuner stores what it picks."""
import numpy as np
import pytest
import torch

from paper_2001_06111_amd import binding, synth
from tests import graphs
from tests.gpu_util import oracle_all, upload

pytestmark = pytest.mark.gpu

DEFAULTS = {"hash_max_work": 2048, "dense_chunk": 6144, "wedge_wg_per_cu": 2, "peel_blocks": 0,
            "active_min": 16384}
# Extremes: every start vertex dense in ranges of 64, one sweep workgroup per
# CU, an 8-workgroup peel rebuilding an active set of one edge.
EXTREMES = [
    dict(DEFAULTS, hash_max_work=1, dense_chunk=64),
    dict(DEFAULTS, hash_max_work=512, dense_chunk=2048, wedge_wg_per_cu=1),
    dict(DEFAULTS, peel_blocks=8, active_min=1),
    dict(DEFAULTS, peel_blocks=100, active_min=1000, wedge_wg_per_cu=7),
]


@pytest.fixture(autouse=True)
def clean_table():
    binding.bt_tune_reset()
    yield
    binding.bt_tune_reset()


def test_results_independent_of_parameters():
    gs = [graphs.worked_example(True)[0], graphs.k2_1001(), synth.complete(7, 9),
          synth.scaled_chunglu(20_000, seed=3), synth.plain_uniform_10k()]
    want = [oracle_all(g) for g in gs]
    for p in EXTREMES:
        binding.bt_tune_reset()
        for g in gs:
            binding.bt_tune_set(g.m, p)
        for g, (osup, obf, ophi) in zip(gs, want):
            sup, phi, st = binding.bt_decompose(upload(g), stats=True)
            assert np.array_equal(sup.cpu().numpy(), osup), (g.name, p)
            assert np.array_equal(phi.cpu().numpy(), ophi), (g.name, p)
            assert st["butterflies"] == obf


def test_batch_independent_of_parameters():
    gs = [synth.batch_graph(i) for i in range(24)]
    dgs = [upload(g) for g in gs]
    ref = [binding.bt_decompose(d)[1].cpu().numpy() for d in dgs]
    total = sum(g.m for g in gs)
    for p in EXTREMES:
        binding.bt_tune_reset()
        binding.bt_tune_set(total, p, batch=True)
        _, phis, _ = binding.bt_decompose_batch(dgs, stats=True)
        for r, ph in zip(ref, phis):
            assert np.array_equal(r, ph.cpu().numpy()), p


def test_autotune_stores_valid_parameters():
    g = synth.scaled_chunglu(200_000, seed=3)
    dg = upload(g)
    osup, _, ophi = oracle_all(g)
    got = binding.bt_tune(dg)
    assert got == binding.bt_tune_get(g.m)
    assert 1 <= got["hash_max_work"] <= 2048 and 64 <= got["dense_chunk"] <= 6144
    assert got["wedge_wg_per_cu"] >= 1 and got["peel_blocks"] >= 0 and got["active_min"] >= 1
    sup, phi, _ = binding.bt_decompose(dg)
    assert np.array_equal(sup.cpu().numpy(), osup) and np.array_equal(phi.cpu().numpy(), ophi)
    gb = [upload(synth.batch_graph(i)) for i in range(8)]
    gotb = binding.bt_tune(gb, binding.BT_TUNE_PEEL)
    assert gotb == binding.bt_tune_get(sum(d.m for d in gb), batch=True)
    with pytest.raises(binding.BtError):
        binding.bt_tune(dg, what=8)
