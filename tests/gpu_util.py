"""Helpers shared by the GPU tests: run through the C ABI, compare with the oracle."""
import numpy as np
import torch

import oracle
from oracle import index_def
from paper_2001_06111_amd import binding


def upload(g):
    return binding.DeviceGraph.upload(g, "cuda")


def gpu_decompose(g, stats=False):
    dg = upload(g)
    sup, phi, st = binding.bt_decompose(dg, stats=stats)
    torch.cuda.synchronize()
    return sup.cpu().numpy(), phi.cpu().numpy(), st


def oracle_all(g):
    sup, bf, pairs = oracle.support(g.n_upper, g.n_lower, g.row_ptr, g.col)
    phi, st = oracle.bitruss(g.n_upper, g.n_lower, g.row_ptr, g.col, sup=sup)
    return sup, bf, phi


def canonical_gpu_index(g, ex):
    """GPU index export -> sorted (x, z, ((e_xy, e_zy) sorted by y)) with global ids."""
    u, v = g.edges()
    nl = g.n_lower
    out = []
    woff = ex["bloom_woff"]
    for b in range(len(woff) - 1):
        pairs = []
        x = z = None
        for w in range(int(woff[b]), int(woff[b + 1])):
            ea, eb = int(ex["wedge_ea"][w]), int(ex["wedge_eb"][w])
            if u[ea] == u[eb]:            # middle vertex is upper
                y = nl + int(u[ea]); xx = int(v[ea]); zz = int(v[eb])
            else:
                assert v[ea] == v[eb]
                y = int(v[ea]); xx = nl + int(u[ea]); zz = nl + int(u[eb])
            assert x is None or (x, z) == (xx, zz)
            x, z = xx, zz
            pairs.append((y, ea, eb))
        pairs.sort()
        out.append((x, z, tuple((ea, eb) for _, ea, eb in pairs)))
    out.sort()
    return out


def check_links(g, ex):
    """Edge-to-wedge links (Section IV, Definitions 8-9; the transpose built by
    the last step of Algorithm 3): edge e links exactly the wedges holding it,
    once each, so the links of all edges are every wedge twice."""
    m = g.m
    ea, eb = ex["wedge_ea"].astype(np.int64), ex["wedge_eb"].astype(np.int64)
    nw = ea.shape[0]
    off, link = ex["link_off"], ex["link"]
    assert off[0] == 0 and off[m] == 2 * nw and np.all(np.diff(off) >= 0)
    want = [[] for _ in range(m)]
    for w in range(nw):
        want[ea[w]].append(w)
        want[eb[w]].append(w)
    for e in range(m):
        assert sorted(link[off[e]:off[e + 1]].tolist()) == sorted(want[e]), e


def check_index(g, ex):
    want = index_def.blooms(g.n_upper, g.n_lower, g.row_ptr, g.col)
    got = canonical_gpu_index(g, ex)
    assert got == want
    check_links(g, ex)
