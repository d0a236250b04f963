"""Python binding of libbt.so: argument marshalling only.

Each function has the name of the C entry point it calls and takes torch
tensors that already live on the GPU (PyTorch is used for device memory and
streams; all compute runs in the library's HIP kernels).  The binding fails
loudly when the library is missing: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbt.so")

BT_OK, BT_EINVAL, BT_ENOMEM, BT_EOVERFLOW, BT_EDEVICE, BT_EBUSY = range(6)
_NAMES = {1: "BT_EINVAL", 2: "BT_ENOMEM", 3: "BT_EOVERFLOW", 4: "BT_EDEVICE", 5: "BT_EBUSY"}


class BtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class bt_csr(ctypes.Structure):
    _fields_ = [("n_upper", ctypes.c_int32), ("n_lower", ctypes.c_int32),
                ("m", ctypes.c_int64), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class bt_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "butterflies", "wedges_po", "blooms", "bloom_wedges", "index_bytes", "levels",
        "rounds", "max_phi", "support_updates", "bloom_visits")] + [
        (n, ctypes.c_float) for n in ("ms_prepare", "ms_count", "ms_link", "ms_peel",
                                      "ms_peel_kernel")] + [
        ("peel_launches", ctypes.c_int32), ("passes", ctypes.c_int32),
        ("support_updates_unbatched", ctypes.c_int64), ("wedge_visits", ctypes.c_int64),
        ("peel_yields", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class bt_index_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "m", "blooms", "bloom_wedges", "links", "butterflies", "wedges_po", "bytes")]


class bt_tune_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "hash_max_work", "dense_chunk", "wedge_wg_per_cu", "peel_blocks", "active_min")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


BT_TUNE_INDEX, BT_TUNE_PEEL = 1, 2

EXPORTED = ["bt_support", "bt_index_build", "bt_index_info_get", "bt_index_export",
            "bt_index_free", "bt_decompose", "bt_decompose_variant", "bt_decompose_pc",
            "bt_decompose_batch",
            "bt_bitruss_components", "bt_release_workspace", "bt_tune", "bt_tune_get",
            "bt_tune_set", "bt_tune_reset", "bt_tune_save", "bt_tune_load",
            "bt_set_allocator", "bt_support_noalloc", "bt_decompose_trace", "bt_last_error",
            "bt_version"]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)

_lib = None


def load():
    """Open libbt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.bt_support.argtypes = [ctypes.POINTER(bt_csr), p, ctypes.POINTER(i64), p]
        L.bt_support_noalloc.argtypes = [ctypes.POINTER(bt_csr), p, ctypes.POINTER(i64), p]
        L.bt_index_build.argtypes = [ctypes.POINTER(bt_csr), ctypes.POINTER(p), p]
        L.bt_index_info_get.argtypes = [p, ctypes.POINTER(bt_index_info)]
        L.bt_index_export.argtypes = [p, p, p, p, p, p, p]
        L.bt_index_free.argtypes = [p]
        L.bt_index_free.restype = None
        L.bt_decompose.argtypes = [ctypes.POINTER(bt_csr), p, p, ctypes.POINTER(bt_stats), p]
        L.bt_decompose_variant.argtypes = [ctypes.POINTER(bt_csr), i32, p, p,
                                           ctypes.POINTER(bt_stats), p]
        L.bt_decompose_pc.argtypes = [ctypes.POINTER(bt_csr), ctypes.c_double, p, p,
                                      ctypes.POINTER(bt_stats), p]
        L.bt_decompose_trace.argtypes = [ctypes.POINTER(bt_csr), p, i32, ctypes.POINTER(i32),
                                         p, p, p, i64, ctypes.POINTER(i64), p, p, p, p]
        L.bt_bitruss_components.argtypes = [ctypes.POINTER(bt_csr), p, i64, p,
                                            ctypes.POINTER(i64), p]
        L.bt_decompose_batch.argtypes = [ctypes.POINTER(bt_csr), i32, ctypes.POINTER(p),
                                         ctypes.POINTER(p), ctypes.POINTER(bt_stats), p]
        L.bt_tune.argtypes = [ctypes.POINTER(bt_csr), i32, ctypes.c_uint32,
                              ctypes.POINTER(bt_tune_params), p]
        L.bt_tune_get.argtypes = [i32, i64, ctypes.POINTER(bt_tune_params)]
        L.bt_tune_set.argtypes = [i32, i64, ctypes.POINTER(bt_tune_params)]
        L.bt_tune_reset.argtypes = []
        L.bt_tune_save.argtypes = [ctypes.c_char_p]
        L.bt_tune_load.argtypes = [ctypes.c_char_p]
        L.bt_release_workspace.restype = None
        L.bt_set_allocator.argtypes = [ALLOC_FN, FREE_FN, p]
        L.bt_set_allocator.restype = ctypes.c_int
        L.bt_last_error.restype = ctypes.c_char_p
        L.bt_version.restype = ctypes.c_char_p
        for name in ("bt_support", "bt_support_noalloc", "bt_decompose_trace", "bt_index_build", "bt_index_info_get", "bt_index_export",
                     "bt_decompose", "bt_decompose_variant", "bt_decompose_pc",
                     "bt_decompose_batch",
                     "bt_bitruss_components", "bt_tune", "bt_tune_get", "bt_tune_set",
                     "bt_tune_reset", "bt_tune_save", "bt_tune_load"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
        atexit.register(_teardown)
    return _lib


def _teardown():
    """At interpreter exit, in order: stop live engines, free the cached
    workspace, forget tuned entries, restore the default allocator (a Python
    hook must not be called once the interpreter is finalising)."""
    L = _lib
    if L is None:
        return
    for e in list(_ENGINES):
        try:
            e.bt_engine_destroy()
        except Exception:
            pass
    try:
        L.bt_release_workspace()
        L.bt_tune_reset()
        L.bt_set_allocator(ALLOC_FN(), FREE_FN(), None)
    except Exception:
        pass


_ENGINES = weakref.WeakSet()
# Every pair of Python callbacks ever installed: a block stays tied to the
# hook that allocated it, so its callbacks must outlive the block.
_CALLBACKS = []


def bt_set_allocator(alloc=None, free=None):
    """Route the library's device allocations through Python callables:
    alloc(nbytes) -> device address (int) or 0/None on failure, and
    free(address, nbytes).  bt_set_allocator() restores hipMalloc/hipFree."""
    L = load()
    if alloc is None and free is None:
        _check(L.bt_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return

    def _a(nbytes, ctx):
        try:
            return alloc(int(nbytes)) or None
        except Exception:
            return None

    def _f(ptr, nbytes, ctx):
        try:
            free(int(ptr), int(nbytes))
        except Exception:
            pass
    cb = (ALLOC_FN(_a), FREE_FN(_f))
    _CALLBACKS.append(cb)
    _check(L.bt_set_allocator(cb[0], cb[1], None))


def use_torch_allocator(device=None):
    """Let PyTorch's caching allocator own the library's device memory."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    idx = dev.index if dev.index is not None else torch.cuda.current_device()

    def alloc(nbytes):
        return torch.cuda.caching_allocator_alloc(nbytes, device=idx)

    def free(ptr, nbytes):
        torch.cuda.caching_allocator_delete(ptr)
    bt_set_allocator(alloc, free)


def _check(rc: int):
    if rc != BT_OK:
        raise BtError(rc, load().bt_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


class DeviceGraph:
    """A graph in device memory: upper-major CSR as torch tensors."""

    def __init__(self, n_upper: int, n_lower: int, row_ptr: torch.Tensor, col: torch.Tensor):
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32
        assert row_ptr.is_cuda and col.is_cuda
        self.n_upper, self.n_lower = int(n_upper), int(n_lower)
        self.row_ptr, self.col = row_ptr.contiguous(), col.contiguous()

    @property
    def m(self) -> int:
        return int(self.col.numel())

    @classmethod
    def upload(cls, g, device="cuda"):
        """From any object with n_upper, n_lower, row_ptr, col (numpy)."""
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int64)).to(device)
        c = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.int32)).to(device)
        return cls(g.n_upper, g.n_lower, rp, c)

    def csr(self) -> bt_csr:
        return bt_csr(self.n_upper, self.n_lower, self.m, self.row_ptr.data_ptr(),
                      self.col.data_ptr() if self.m > 0 else 0)


def bt_support(g: DeviceGraph, stream=None):
    """(int64 supports on the device, total butterflies)."""
    L = load()
    sup = torch.empty(g.m, dtype=torch.int64, device=g.col.device)
    bf = ctypes.c_int64(0)
    c = g.csr()
    _check(L.bt_support(ctypes.byref(c), _ptr(sup), ctypes.byref(bf), _stream(stream)))
    return sup, int(bf.value)


def bt_support_noalloc(g: DeviceGraph, out_sup: torch.Tensor | None = None, stream=None):
    """bt_support from static scratch: (supports, total butterflies).  Pass
    `out_sup` (int64[m] on the device) for a call that allocates nothing."""
    L = load()
    sup = out_sup if out_sup is not None else torch.empty(g.m, dtype=torch.int64,
                                                          device=g.col.device)
    bf = ctypes.c_int64(0)
    c = g.csr()
    _check(L.bt_support_noalloc(ctypes.byref(c), _ptr(sup), ctypes.byref(bf), _stream(stream)))
    return sup, int(bf.value)


def bt_decompose(g: DeviceGraph, want_sup: bool = True, stats: bool = False, stream=None,
                 out_phi: torch.Tensor | None = None, out_sup: torch.Tensor | None = None):
    """(supports or None, bitruss numbers, stats dict or None)."""
    L = load()
    dev = g.col.device
    phi = out_phi if out_phi is not None else torch.empty(g.m, dtype=torch.int64, device=dev)
    sup = out_sup if out_sup is not None else (
        torch.empty(g.m, dtype=torch.int64, device=dev) if want_sup else None)
    st = bt_stats()
    c = g.csr()
    _check(L.bt_decompose(ctypes.byref(c), _ptr(sup), _ptr(phi),
                          ctypes.byref(st) if stats else None, _stream(stream)))
    return sup, phi, (st.as_dict() if stats else None)


def bt_tune(graphs, what: int = BT_TUNE_INDEX | BT_TUNE_PEEL, stream=None) -> dict:
    """Autotune launch parameters on one DeviceGraph (single-graph calls) or a
    list of them (batches); returns the stored parameters."""
    L = load()
    gl = graphs if isinstance(graphs, (list, tuple)) else [graphs]
    arr = (bt_csr * len(gl))(*[g.csr() for g in gl])
    out = bt_tune_params()
    _check(L.bt_tune(arr, len(gl), ctypes.c_uint32(what), ctypes.byref(out), _stream(stream)))
    return out.as_dict()


def bt_tune_get(m: int, batch: bool = False) -> dict:
    out = bt_tune_params()
    _check(load().bt_tune_get(int(batch), int(m), ctypes.byref(out)))
    return out.as_dict()


def bt_tune_set(m: int, params: dict, batch: bool = False):
    p = bt_tune_params(**{k: int(v) for k, v in params.items()})
    _check(load().bt_tune_set(int(batch), int(m), ctypes.byref(p)))


def bt_tune_reset():
    _check(load().bt_tune_reset())


def bt_tune_save(path: str):
    _check(load().bt_tune_save(os.fsencode(path)))


def bt_tune_load(path: str):
    _check(load().bt_tune_load(os.fsencode(path)))


BT_PEEL_BATCH_BLOOM, BT_PEEL_BATCH_EDGE, BT_PEEL_AUTO = 0, 1, 2


def bt_decompose_variant(g: DeviceGraph, variant: int, want_sup: bool = True,
                         stats: bool = False, stream=None):
    """bt_decompose with a chosen peel variant (BT_PEEL_*): (supports or None,
    bitruss numbers, stats dict or None)."""
    L = load()
    dev = g.col.device
    phi = torch.empty(g.m, dtype=torch.int64, device=dev)
    sup = torch.empty(g.m, dtype=torch.int64, device=dev) if want_sup else None
    st = bt_stats()
    c = g.csr()
    _check(L.bt_decompose_variant(ctypes.byref(c), ctypes.c_int32(int(variant)), _ptr(sup),
                                  _ptr(phi), ctypes.byref(st) if stats else None,
                                  _stream(stream)))
    return sup, phi, (st.as_dict() if stats else None)


def bt_decompose_trace(g: DeviceGraph, max_rounds: int = 256, max_wedges: int = 1 << 16,
                       stream=None):
    """Round-by-round trace of the peel (small graphs): dict with phi (device
    tensor), level[k], removed[k, m] (bool), sup[k, m], wedge_ea, wedge_eb and
    wedge_k[k, w] (numpy)."""
    L = load()
    m = g.m
    phi = torch.empty(m, dtype=torch.int64, device=g.col.device)
    lv = np.zeros(max_rounds, np.int32)
    rm = np.zeros((max_rounds, m), np.int8)
    sp = np.zeros((max_rounds, m), np.int64)
    ea = np.zeros(max_wedges, np.int32)
    eb = np.zeros(max_wedges, np.int32)
    wk = np.zeros((max_rounds, max_wedges), np.int32)
    nr, nw = ctypes.c_int32(0), ctypes.c_int64(0)

    def p(a):
        return a.ctypes.data_as(ctypes.c_void_p)
    c = g.csr()
    _check(L.bt_decompose_trace(ctypes.byref(c), _ptr(phi), max_rounds, ctypes.byref(nr), p(lv),
                                p(rm), p(sp), max_wedges, ctypes.byref(nw), p(ea), p(eb), p(wk),
                                _stream(stream)))
    k, w = nr.value, nw.value
    return {"phi": phi, "level": lv[:k], "removed": rm[:k].astype(bool), "sup": sp[:k],
            "wedge_ea": ea[:w], "wedge_eb": eb[:w], "wedge_k": wk[:k, :w]}


def bt_decompose_pc(g: DeviceGraph, tau: float = 0.1, want_sup: bool = True, stats: bool = False,
                    stream=None, out_phi: torch.Tensor | None = None,
                    out_sup: torch.Tensor | None = None):
    """BiT-PC: (supports or None, bitruss numbers, stats dict or None)."""
    L = load()
    dev = g.col.device
    phi = out_phi if out_phi is not None else torch.empty(g.m, dtype=torch.int64, device=dev)
    sup = out_sup if out_sup is not None else (
        torch.empty(g.m, dtype=torch.int64, device=dev) if want_sup else None)
    st = bt_stats()
    c = g.csr()
    _check(L.bt_decompose_pc(ctypes.byref(c), ctypes.c_double(tau), _ptr(sup), _ptr(phi),
                             ctypes.byref(st) if stats else None, _stream(stream)))
    return sup, phi, (st.as_dict() if stats else None)


def bt_bitruss_components(g: DeviceGraph, phi: torch.Tensor, k: int, stream=None):
    """(int32 component of every edge of the k-bitruss, -1 elsewhere; count)."""
    L = load()
    assert phi.dtype == torch.int64 and phi.numel() == g.m
    comp = torch.empty(g.m, dtype=torch.int32, device=g.col.device)
    n = ctypes.c_int64(0)
    c = g.csr()
    _check(L.bt_bitruss_components(ctypes.byref(c), _ptr(phi), ctypes.c_int64(int(k)), _ptr(comp),
                                   ctypes.byref(n), _stream(stream)))
    return comp, int(n.value)


def bt_decompose_batch(graphs, want_sup: bool = True, stats: bool = False, stream=None):
    """Lists of supports and bitruss numbers (device tensors), plus summed stats."""
    L = load()
    n = len(graphs)
    dev = graphs[0].col.device if n else "cuda"
    phis = [torch.empty(g.m, dtype=torch.int64, device=dev) for g in graphs]
    sups = [torch.empty(g.m, dtype=torch.int64, device=dev) for g in graphs] if want_sup else None
    arr = (bt_csr * max(n, 1))(*[g.csr() for g in graphs])
    pp = (ctypes.c_void_p * max(n, 1))(*[_ptr(t).value or 0 for t in phis])
    sp = (ctypes.c_void_p * max(n, 1))(*[_ptr(t).value or 0 for t in sups]) if want_sup else None
    st = bt_stats()
    _check(L.bt_decompose_batch(arr, n, sp, pp, ctypes.byref(st) if stats else None,
                                _stream(stream)))
    return sups, phis, (st.as_dict() if stats else None)


class BtIndex:
    """Handle of a device-resident BE-Index (bt_index_build / bt_index_free)."""

    def __init__(self, handle, m: int):
        self._h = handle
        self.m = m

    def info(self) -> dict:
        info = bt_index_info()
        _check(load().bt_index_info_get(self._h, ctypes.byref(info)))
        return {n: getattr(info, n) for n, _ in info._fields_}

    def export(self) -> dict:
        """Host copies: bloom_woff, wedge_ea, wedge_eb, link_off, link, sup (numpy)."""
        inf = self.info()
        nb, nw = inf["blooms"], inf["bloom_wedges"]
        out = dict(bloom_woff=np.zeros(nb + 1, np.int64), wedge_ea=np.zeros(nw, np.int32),
                   wedge_eb=np.zeros(nw, np.int32), link_off=np.zeros(self.m + 1, np.int64),
                   link=np.zeros(2 * nw, np.int64), sup=np.zeros(self.m, np.int64))

        def p(a):
            return a.ctypes.data_as(ctypes.c_void_p)
        _check(load().bt_index_export(self._h, p(out["bloom_woff"]), p(out["wedge_ea"]),
                                      p(out["wedge_eb"]), p(out["link_off"]), p(out["link"]),
                                      p(out["sup"])))
        return out

    def free(self):
        if self._h:
            load().bt_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def bt_index_build(g: DeviceGraph, stream=None) -> BtIndex:
    L = load()
    h = ctypes.c_void_p(0)
    c = g.csr()
    _check(L.bt_index_build(ctypes.byref(c), ctypes.byref(h), _stream(stream)))
    return BtIndex(h, g.m)


def bt_release_workspace():
    load().bt_release_workspace()


def bt_version() -> str:
    return load().bt_version().decode()


# --- serving engine ----------------------------------------------------------

EXPORTED += ["bt_engine_create", "bt_engine_submit", "bt_engine_step", "bt_engine_poll",
             "bt_engine_drain", "bt_engine_stats", "bt_engine_memory", "bt_engine_destroy"]


def _engine_lib():
    L = load()
    if not getattr(L, "_engine_ready", False):
        p, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.bt_engine_create.argtypes = [i64, i32, i32, ctypes.POINTER(p)]
        L.bt_engine_submit.argtypes = [p, ctypes.POINTER(bt_csr), p, p, u64]
        L.bt_engine_poll.argtypes = [p, ctypes.POINTER(u64), ctypes.POINTER(i32), i32,
                                     ctypes.POINTER(i32)]
        L.bt_engine_step.argtypes = [p, ctypes.POINTER(i32)]
        L.bt_engine_drain.argtypes = [p]
        L.bt_engine_stats.argtypes = [p] + [ctypes.POINTER(i64)] * 4
        L.bt_engine_memory.argtypes = [p] + [ctypes.POINTER(i64)] * 4
        L.bt_engine_destroy.argtypes = [p]
        L.bt_engine_destroy.restype = None
        for n in ("bt_engine_create", "bt_engine_submit", "bt_engine_step", "bt_engine_poll",
                  "bt_engine_drain", "bt_engine_stats", "bt_engine_memory"):
            getattr(L, n).restype = ctypes.c_int
        L._engine_ready = True
    return L


class BtEngine:
    """bt_engine_* handle.  Keeps each request's graph and outputs alive until
    it completes; results are device tensors."""

    def __init__(self, hbm_budget: int = 0, slots: int = 0, max_batch: int = 1024):
        L = _engine_lib()
        self._h = ctypes.c_void_p(0)
        _check(L.bt_engine_create(int(hbm_budget), int(slots), int(max_batch),
                                  ctypes.byref(self._h)))
        self._live = {}
        self.results = {}
        _ENGINES.add(self)

    def bt_engine_submit(self, g: DeviceGraph, req_id: int, want_sup: bool = False):
        L = _engine_lib()
        dev = g.col.device
        phi = torch.empty(g.m, dtype=torch.int64, device=dev)
        sup = torch.empty(g.m, dtype=torch.int64, device=dev) if want_sup else None
        c = g.csr()
        # the engine reads the graph on its own streams: finish pending uploads
        torch.cuda.current_stream().synchronize()
        self._live[req_id] = (g, sup, phi)  # before submit: it may complete at once
        rc = L.bt_engine_submit(self._h, ctypes.byref(c), _ptr(sup), _ptr(phi),
                                ctypes.c_uint64(req_id))
        if rc != BT_OK:
            self._live.pop(req_id, None)
        _check(rc)

    def bt_engine_poll(self, cap: int = 4096):
        """Completed (id, status) pairs; their (sup, phi) move to self.results."""
        L = _engine_lib()
        ids = (ctypes.c_uint64 * cap)()
        st = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32(0)
        _check(L.bt_engine_poll(self._h, ids, st, cap, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            rid, s = int(ids[i]), int(st[i])
            g, sup, phi = self._live.pop(rid)
            self.results[rid] = (s, sup, phi)
            out.append((rid, s))
        return out

    def bt_engine_step(self):
        """Caller-driven engines (slots=-1): run one batch on this thread;
        returns how many requests it completed (0: none queued)."""
        n = ctypes.c_int32(0)
        _check(_engine_lib().bt_engine_step(self._h, ctypes.byref(n)))
        return n.value

    def bt_engine_drain(self):
        _check(_engine_lib().bt_engine_drain(self._h))

    def bt_engine_stats(self):
        b, a, q, y = (ctypes.c_int64(0) for _ in range(4))
        _check(_engine_lib().bt_engine_stats(self._h, ctypes.byref(b), ctypes.byref(a),
                                             ctypes.byref(q), ctypes.byref(y)))
        return {"batches": b.value, "admitted": a.value, "queued": q.value,
                "peel_yields": y.value}

    def bt_engine_memory(self):
        v = [ctypes.c_int64(0) for _ in range(4)]
        _check(_engine_lib().bt_engine_memory(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("budget", "held", "peak_held", "peak_committed"), (x.value for x in v)))

    def bt_engine_destroy(self):
        if self._h:
            _engine_lib().bt_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.bt_engine_destroy()
        except Exception:
            pass
