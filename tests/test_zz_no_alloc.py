"""bt_support_noalloc (static scratch, no device allocation) against
bt_support, through the C ABI on the GPU."""
import numpy as np
import pytest
import torch

from paper_2001_06111_amd import binding, synth
from tests.gpu_util import oracle_all, upload

pytestmark = pytest.mark.gpu


def _pair(g):
    dg = upload(g)
    sup, bf = binding.bt_support(dg)
    out = torch.full((g.m,), -7, dtype=torch.int64, device="cuda")
    sup2, bf2 = binding.bt_support_noalloc(dg, out_sup=out)
    torch.cuda.synchronize()
    return sup, bf, sup2, bf2


def test_noalloc_equals_support_twice_smaller_second():
    a = synth.scaled_chunglu(150_000, seed=21)
    b = synth.batch_graph(3)
    assert b.m < a.m
    for g in (a, b):
        sup, bf, sup2, bf2 = _pair(g)
        assert torch.equal(sup, sup2) and bf == bf2
    osup, obf, _ = oracle_all(b)
    assert np.array_equal(sup2.cpu().numpy(), osup) and bf2 == obf


def test_noalloc_allocates_nothing():
    g = synth.batch_graph(11)
    dg = upload(g)
    out = torch.empty(g.m, dtype=torch.int64, device="cuda")
    binding.bt_support_noalloc(dg, out_sup=out)  # first call on this device
    seen = []

    def alloc(n):
        seen.append(n)
        return torch.cuda.caching_allocator_alloc(n)

    binding.bt_set_allocator(alloc, lambda p, n: torch.cuda.caching_allocator_delete(p))
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        sup, bf = binding.bt_support_noalloc(dg, out_sup=out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
    finally:
        binding.bt_set_allocator()
    assert seen == []
    ref, rbf = binding.bt_support(dg)
    assert torch.equal(ref, sup) and rbf == bf


def test_noalloc_size_limits():
    # the largest accepted graph: 2^18 edges over 2^18 vertices
    g = synth.chung_lu(1 << 17, 1 << 17, 1 << 18, 2.1, 2.5, 4096, 4096, 5)
    assert g.m == 1 << 18 and g.n_upper + g.n_lower == 1 << 18
    sup, bf, sup2, bf2 = _pair(g)
    assert torch.equal(sup, sup2) and bf == bf2
    big = synth.scaled_chunglu((1 << 18) + 1, seed=3)
    with pytest.raises(binding.BtError) as ei:
        binding.bt_support_noalloc(upload(big))
    assert ei.value.status == binding.BT_EOVERFLOW
    empty = synth.from_edges(3, 4, [])
    s, b = binding.bt_support_noalloc(upload(empty))
    assert s.numel() == 0 and b == 0
