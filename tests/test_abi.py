"""The C-ABI library loads on the CPU and exports every declared entry point."""
import ctypes
import os
import re

from paper_2001_06111_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bt_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("bt_support", "bt_index_build", "bt_decompose", "bt_decompose_variant",
              "bt_decompose_pc",
              "bt_decompose_batch"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(binding.EXPORTED)


def test_version_without_gpu():
    assert binding.bt_version().startswith("bt-mi355x")
