"""The launch-parameter table and its file format (host only, no GPU)."""
import os

import pytest

from paper_2001_06111_amd import binding

DEFAULTS = {"hash_max_work": 2048, "dense_chunk": 6144, "wedge_wg_per_cu": 2, "peel_blocks": 0,
            "active_min": 16384}


@pytest.fixture(autouse=True)
def clean_table():
    binding.bt_tune_reset()
    yield
    binding.bt_tune_reset()


def test_defaults_and_nearest_class():
    assert binding.bt_tune_get(5_000_000) == DEFAULTS
    p = dict(DEFAULTS, hash_max_work=1024, peel_blocks=128)
    binding.bt_tune_set(5_000_000, p)          # class of 2^22 <= m < 2^23
    assert binding.bt_tune_get(5_000_000) == p
    assert binding.bt_tune_get(4_200_000) == p   # same class
    assert binding.bt_tune_get(100) == p         # nearest tuned class of the kind
    assert binding.bt_tune_get(5_000_000, batch=True) == DEFAULTS  # other kind untouched
    q = dict(DEFAULTS, dense_chunk=2048)
    binding.bt_tune_set(1 << 14, q)
    assert binding.bt_tune_get(1 << 14) == q
    assert binding.bt_tune_get(3_000_000) == p   # class 12 is nearer than class 5
    assert binding.bt_tune_get(200) == q


@pytest.mark.parametrize("bad", [{"hash_max_work": 0}, {"hash_max_work": 4096},
                                 {"dense_chunk": 10}, {"dense_chunk": 7000},
                                 {"wedge_wg_per_cu": 0}, {"peel_blocks": -1},
                                 {"active_min": 0}])
def test_out_of_range_rejected(bad):
    with pytest.raises(binding.BtError) as ei:
        binding.bt_tune_set(1000, dict(DEFAULTS, **bad))
    assert ei.value.status == binding.BT_EINVAL
    assert binding.bt_tune_get(1000) == DEFAULTS


def test_save_load_round_trip(tmp_path):
    a = dict(DEFAULTS, hash_max_work=512, active_min=16384)
    b = dict(DEFAULTS, wedge_wg_per_cu=1, peel_blocks=192)
    binding.bt_tune_set(5_000_000, a)
    binding.bt_tune_set(20_000_000, b, batch=True)
    f = str(tmp_path / "tune.txt")
    binding.bt_tune_save(f)
    lines = open(f).read().split("\n")
    assert lines[0].startswith("bt-tune 1 ")
    binding.bt_tune_reset()
    assert binding.bt_tune_get(5_000_000) == DEFAULTS
    binding.bt_tune_load(f)
    assert binding.bt_tune_get(5_000_000) == a
    assert binding.bt_tune_get(20_000_000, batch=True) == b


@pytest.mark.parametrize("text", [
    "not a tuning file\n",
    "bt-tune 2 unknown\n",
    "bt-tune 1 unknown\nsingle 12 512 6144 2 0\n",            # a field short
    "bt-tune 1 unknown\nsingle 12 9999 6144 2 0 65536\n",     # out of range
    "bt-tune 1 unknown\nsingle 40 512 6144 2 0 65536\n",      # no such class
    "bt-tune 1 unknown\nsome 12 512 6144 2 0 65536\n",        # no such kind
    "bt-tune 1 unknown\nsingle 3 512 6144 2 0 65536\nsingle 12 0 6144 2 0 65536\n",
])
def test_bad_files_change_nothing(tmp_path, text):
    f = tmp_path / "bad.txt"
    f.write_text(text)
    with pytest.raises(binding.BtError) as ei:
        binding.bt_tune_load(str(f))
    assert ei.value.status == binding.BT_EINVAL
    assert binding.bt_tune_get(1 << 13) == DEFAULTS


def test_missing_file():
    with pytest.raises(binding.BtError):
        binding.bt_tune_load(os.path.join("/nonexistent", "tune.txt"))


def test_cache_file_from_environment(tmp_path):
    """BT_TUNE_CACHE names a file that the library loads at its first lookup."""
    import subprocess
    import sys
    f = tmp_path / "tune.txt"
    f.write_text("bt-tune 1 unknown\nsingle 13 1024 4096 1 128 4096\n")
    code = ("import json; from paper_2001_06111_amd import binding; "
            "print(json.dumps(binding.bt_tune_get(5_000_000)))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, BT_TUNE_CACHE=str(f), PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=120, cwd=root)
    assert out.returncode == 0, out.stderr
    import json
    assert json.loads(out.stdout.strip().splitlines()[-1]) == {
        "hash_max_work": 1024, "dense_chunk": 4096, "wedge_wg_per_cu": 1, "peel_blocks": 128,
        "active_min": 4096}
