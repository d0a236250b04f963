"""The pins catch plausible mistakes: each test plants one in a copy of the
oracle's C source, builds it on the CPU and checks that some pin fails."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import api, brute
from paper_2001_06111_amd import synth
from tests import graphs

MUTATIONS = {
    "dropped_minus_one": ("s += (int64_t)cnt[w] - 1;", "s += (int64_t)cnt[w];"),
    "pairs_counted_twice": ("if (w > a) total += c * (c - 1) / 2;", "total += c * (c - 1) / 2;"),
    # Every frontier edge of a butterfly acts on it, not only the smallest.
    "no_butterfly_owner": ("if (in_f[f[j]] && f[j] < e) return 0;", "(void)0;"),
    "frontier_off_by_one": ("if (old > level && old - 1 <= level) {", "if (old > level && old - 1 <= level + 1) {"),
    # A removed edge left in its upper row: walks then count butterflies
    # through edges that are gone.
    "removed_edge_counted": ("rows_remove(&RU, urow[e], e);", "(void)0;"),
    "decrement_by_two": ("int64_t old = __atomic_fetch_sub(&s[f[j]], 1, __ATOMIC_RELAXED);\n        if (old > level && old - 1 <= level) {",
                         "int64_t old = __atomic_fetch_sub(&s[f[j]], 2, __ATOMIC_RELAXED);\n        if (old > level && old - 2 <= level) {"),
}


def _pins_pass(lib):
    """The oracle pins of test_oracle.py, condensed; True if all hold."""
    def sup(g):
        return oracle.support(g.n_upper, g.n_lower, g.row_ptr, g.col, lib=lib)

    def phi(g):
        return oracle.bitruss(g.n_upper, g.n_lower, g.row_ptr, g.col, lib=lib)[0]

    g, nm, fx = graphs.worked_example(True)
    s, bf, pairs = sup(g)
    if any(s[nm[k]] != v for k, v in fx["support"].items()) or bf != 4 or pairs != 4:
        return False
    p = phi(g)
    if any(p[nm[f"e{i}"]] != fx["phi"][f"e{i}"] for i in range(9)):
        return False
    for a, b in [(3, 4), (5, 5)]:
        k = synth.complete(a, b)
        if not np.all(sup(k)[0] == (a - 1) * (b - 1)) or not np.all(phi(k) == (a - 1) * (b - 1)):
            return False
    for seed in range(12):
        g = graphs.random_dense(7, 8, 0.6, seed)
        bs, bb = brute.support(g.n_upper, g.n_lower, g.row_ptr, g.col)
        s, bf, pairs = sup(g)
        if not np.array_equal(s, bs) or bf != bb or pairs != bb:
            return False
        if not np.array_equal(phi(g), brute.bitruss(g.n_upper, g.n_lower, g.row_ptr, g.col)):
            return False
    return True


def test_unmutated_oracle_passes():
    assert _pins_pass(api.load_library(oracle.lib_path()))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.lib_path()), "bt_oracle.c")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) >= 1, "mutation anchor not found"
    mutated = src.replace(old, new)
    c = tmp_path / "mut.c"
    so = tmp_path / f"libmut_{name}.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(c)],
                   check=True)
    assert not _pins_pass(api.load_library(str(so)))
