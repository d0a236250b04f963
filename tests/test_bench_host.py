"""bench.py's host-side measurement helpers, on the CPU: the algorithmic
bytes of a peel, the roofline record built from them, and the rule that a
committed HBM-traffic summary counts only for the kernel sources it was
measured on."""
import hashlib
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


STATS = {"peel_launches": 2, "ms_peel_kernel": 2000.0, "bloom_wedges": 1000,
         "wedge_visits": 5000, "support_updates": 7000}


def test_peel_bytes_formula(bench):
    alg, alg32 = bench.peel_bytes(STATS)
    assert alg == 40 * 2 * 1000 + 41 * 5000
    assert alg32 == 29 * 2 * 1000 + 25 * 5000


def test_roofline_record(bench):
    r = bench.roofline("k", STATS, 4.0e6)
    alg = 40 * 2 * 1000 + 41 * 5000
    assert r["achieved"] == pytest.approx(alg / 2.0 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["avg_launch_ms"] == 1000.0 and r["launches"] == 2
    assert r["traffic"] == 2.0e6  # per launch
    assert r["traffic_gbs"] == pytest.approx(4.0e6 / 2.0 / 1e9)
    assert r["decrements_per_s"] == pytest.approx(3500.0)
    assert bench.roofline("k", STATS, None)["traffic"] is None


def test_measured_traffic_needs_matching_sources(bench, tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2001_06111_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (csrc / "a.hip").write_bytes(b"kernel a")
    (csrc / "b.h").write_bytes(b"header b")
    digest = hashlib.sha256(b"kernel a" + b"header b").hexdigest()
    (tmp_path / "profiles" / "t.md").write_text(
        f"# t\n\n- kernel_source_sha256: {digest}\n- hbm_bytes_total: 123456\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("t.md", ("a.hip", "b.h")) == 123456.0
    assert bench.measured_traffic("t.md", ("b.h", "a.hip")) is None  # order is part of it
    (csrc / "a.hip").write_bytes(b"kernel a, changed")
    assert bench.measured_traffic("t.md", ("a.hip", "b.h")) is None
    assert bench.measured_traffic("missing.md", ("a.hip",)) is None
