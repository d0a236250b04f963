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


def _csr(nu=3, nl=4, m=5, rp=0x1000, col=0x2000):
    return binding.bt_csr(nu, nl, m, rp, col)


def test_argument_errors_without_gpu():
    """Malformed descriptors and arguments are rejected before any device
    work, with the documented status and a message."""
    L = binding._engine_lib()
    P = ctypes.c_void_p
    fake = P(0x3000)
    handle = P(0)
    n = ctypes.c_int32(0)
    cases = [
        (lambda: L.bt_engine_create(0, -2, 0, ctypes.byref(handle)), binding.BT_EINVAL),
        (lambda: L.bt_engine_create(0, 1, -1, ctypes.byref(handle)), binding.BT_EINVAL),
        (lambda: L.bt_engine_step(None, ctypes.byref(n)), binding.BT_EINVAL),
        (lambda: L.bt_engine_poll(None, None, None, 0, ctypes.byref(n)), binding.BT_EINVAL),
        (lambda: L.bt_decompose(None, None, fake, None, None), binding.BT_EINVAL),
        (lambda: L.bt_decompose(ctypes.byref(_csr(m=-1)), None, fake, None, None),
         binding.BT_EINVAL),
        (lambda: L.bt_decompose(ctypes.byref(_csr(nu=-2)), None, fake, None, None),
         binding.BT_EINVAL),
        (lambda: L.bt_decompose(ctypes.byref(_csr(nu=2**31 - 1, nl=1)), None, fake, None, None),
         binding.BT_EOVERFLOW),
        (lambda: L.bt_decompose(ctypes.byref(_csr(m=2**31)), None, fake, None, None),
         binding.BT_EOVERFLOW),
        (lambda: L.bt_decompose(ctypes.byref(_csr(rp=None)), None, fake, None, None),
         binding.BT_EINVAL),
        (lambda: L.bt_decompose(ctypes.byref(_csr(col=None)), None, fake, None, None),
         binding.BT_EINVAL),
        (lambda: L.bt_decompose(ctypes.byref(_csr()), None, None, None, None), binding.BT_EINVAL),
        (lambda: L.bt_decompose_variant(ctypes.byref(_csr()), 5, None, fake, None, None),
         binding.BT_EINVAL),
        (lambda: L.bt_decompose_pc(ctypes.byref(_csr()), ctypes.c_double(0.0), None, fake,
                                   None, None), binding.BT_EINVAL),
        (lambda: L.bt_decompose_pc(ctypes.byref(_csr()), ctypes.c_double(1.5), None, fake,
                                   None, None), binding.BT_EINVAL),
        (lambda: L.bt_decompose_batch(None, -1, None, None, None, None), binding.BT_EINVAL),
        (lambda: L.bt_bitruss_components(ctypes.byref(_csr()), None, 1, fake, None, None),
         binding.BT_EINVAL),
        (lambda: L.bt_tune(ctypes.byref(_csr()), 0, 3, None, None), binding.BT_EINVAL),
        (lambda: L.bt_tune(ctypes.byref(_csr()), 1, 8, None, None), binding.BT_EINVAL),
        (lambda: L.bt_tune_get(0, -1, None), binding.BT_EINVAL),
        (lambda: L.bt_set_allocator(binding.ALLOC_FN(), binding.FREE_FN(lambda p, n, c: None),
                                    None), binding.BT_EINVAL),
        (lambda: L.bt_set_allocator(binding.ALLOC_FN(lambda n, c: None), binding.FREE_FN(),
                                    None), binding.BT_EINVAL),
    ]
    for i, (call, want) in enumerate(cases):
        rc = call()
        msg = L.bt_last_error().decode()
        assert rc == want, (i, rc, msg)
        assert msg, i
