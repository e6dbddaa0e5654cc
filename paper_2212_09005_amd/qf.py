"""Python binding of libqf.so (include/qf.h): the same calls, marshalled with ctypes.

Only argument marshalling happens here: every step of insert / query / count /
delete runs in the library's HIP kernels on the device that holds the tensors.
PyTorch supplies device memory and streams.  If libqf.so has not been built,
loading fails with an error instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libqf.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "qf.h")

QF_OK = 0
QF_ERR_ARG = -1
QF_ERR_FULL = -2
QF_ERR_OOM = -3
QF_ERR_DEVICE = -4
QF_ERR_COUNT_OVERFLOW = -5
QF_ERR_STALLED = -6
QF_ERR_BUDGET = -7
QF_ERR_LIMIT = -8
NOALLOC_MAX_KEYS = 1 << 19
ERRORS = {
    QF_ERR_ARG: "QF_ERR_ARG",
    QF_ERR_FULL: "QF_ERR_FULL",
    QF_ERR_OOM: "QF_ERR_OOM",
    QF_ERR_DEVICE: "QF_ERR_DEVICE",
    QF_ERR_COUNT_OVERFLOW: "QF_ERR_COUNT_OVERFLOW",
    QF_ERR_STALLED: "QF_ERR_STALLED",
    QF_ERR_BUDGET: "QF_ERR_BUDGET",
    QF_ERR_LIMIT: "QF_ERR_LIMIT",
}


class QFError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"{what}: {ERRORS.get(code, code)}")
        self.code = code


class _Tuning(ctypes.Structure):
    _fields_ = [
        ("region_log2", ctypes.c_uint32),
        ("sort_tile", ctypes.c_uint32),
        ("sort_chunk", ctypes.c_uint32),
        ("lookup_keys_per_lane", ctypes.c_uint32),
    ]


TUNING_FIELDS = ("region_log2", "sort_tile", "sort_chunk", "lookup_keys_per_lane")


def _tuning(d: dict) -> _Tuning:
    bad = set(d) - set(TUNING_FIELDS)
    if bad:
        raise ValueError(f"unknown tuning fields {sorted(bad)}")
    return _Tuning(*[int(d.get(k, 0)) for k in TUNING_FIELDS])


def _tuning_dict(t: _Tuning) -> dict:
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}


class _Layout(ctypes.Structure):
    _fields_ = [
        ("header", ctypes.c_uint64 * 8),
        ("occ_words", ctypes.c_void_p),
        ("runend_words", ctypes.c_void_p),
        ("slots", ctypes.c_void_p),
        ("offsets", ctypes.c_void_p),
    ]


@dataclass
class QFLayout:
    """Logical table as host arrays (see qf_layout_t in include/qf.h)."""

    occ_words: np.ndarray  # uint64[N/64]
    runend_words: np.ndarray  # uint64[P/64]
    slots: np.ndarray  # uint16[P]
    offsets: np.ndarray  # uint32[P/64]
    header: np.ndarray  # uint64[8]


_lib = None


def declared_functions() -> list[str]:
    """Names of the functions include/qf.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qf_[a-z0-9_]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with paper_2212_09005_amd/build.py "
            "(or __graft_entry__.build()); there is no fallback implementation"
        )
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "qf_create": (vp, [u32, u32]),
        "qf_destroy": (None, [vp]),
        "qf_insert_batch": (i32, [vp, vp, u64, vp]),
        "qf_insert_batch_noalloc": (i32, [vp, vp, u64, vp]),
        "qf_stats": (i32, [vp, ctypes.POINTER(ctypes.c_uint64), vp]),
        "qf_enumerate": (i32, [vp, vp, vp, u64, ctypes.POINTER(ctypes.c_uint64), vp]),
        "qf_merge_into": (i32, [vp, vp, i32, vp, vp]),
        "qf_resize": (vp, [vp, u32, u32, vp]),
        "qf_query_batch": (i32, [vp, vp, u64, vp, vp]),
        "qf_count_batch": (i32, [vp, vp, u64, vp, vp]),
        "qf_delete_batch": (i32, [vp, vp, u64, vp, vp]),
        "qf_point_insert": (i32, [vp, vp, u64, vp, vp]),
        "qf_create_kv": (vp, [u32, u32, u32]),
        "qf_kv_insert_batch": (i32, [vp, vp, vp, u64, vp]),
        "qf_kv_delete_batch": (i32, [vp, vp, vp, u64, vp, vp]),
        "qf_kv_lookup_batch": (i32, [vp, vp, u64, vp, vp, vp]),
        "qf_point_delete": (i32, [vp, vp, u64, vp, vp, vp]),
        "qf_sync": (i32, [vp, vp]),
        "qf_export": (i32, [vp, ctypes.POINTER(_Layout), vp]),
        "qf_import": (i32, [vp, ctypes.POINTER(_Layout), vp]),
        "qf_last_error": (i32, []),
        "qf_table_bytes": (u64, [u32, u32]),
        "qf_info": (i32, [vp, ctypes.POINTER(ctypes.c_uint64)]),
        "qf_profile_enable": (i32, [vp, i32]),
        "qf_profile_read": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)]),
        "qf_reserve": (i32, [vp, u64, vp]),
        "qf_set_reserve": (i32, [vp, u64, vp]),
        "qf_set_create": (vp, [ctypes.POINTER(vp), u32]),
        "qf_set_destroy": (None, [vp]),
        "qf_set_insert_batch": (i32, [vp, vp, vp, u64, vp]),
        "qf_set_delete_batch": (i32, [vp, vp, vp, u64, vp, vp]),
        "qf_set_query_batch": (i32, [vp, vp, vp, u64, vp, vp]),
        "qf_set_count_batch": (i32, [vp, vp, vp, u64, vp, vp]),
        "qf_set_sync": (i32, [vp, vp]),
        "qf_set_info": (i32, [vp, ctypes.POINTER(ctypes.c_uint64)]),
        "qf_set_profile_enable": (i32, [vp, i32]),
        "qf_set_profile_read": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)]),
        "qf_set_errors": (i32, [vp, ctypes.POINTER(ctypes.c_int32), vp]),
        "qf_set_insert_some": (i32, [vp, ctypes.POINTER(ctypes.c_uint32), u32, vp, vp, u64, vp]),
        "qf_set_delete_some": (i32, [vp, ctypes.POINTER(ctypes.c_uint32), u32, vp, vp, u64, vp, vp]),
        "qf_tune": (i32, [vp, ctypes.POINTER(_Tuning)]),
        "qf_get_tuning": (i32, [vp, ctypes.POINTER(_Tuning)]),
        "qf_set_tune": (i32, [vp, ctypes.POINTER(_Tuning)]),
        "qf_set_get_tuning": (i32, [vp, ctypes.POINTER(_Tuning)]),
        "qf_autotune_set": (i32, [ctypes.POINTER(ctypes.c_uint32), u32, u32, ctypes.c_double, u64,
                                  ctypes.POINTER(_Tuning), ctypes.POINTER(ctypes.c_double)]),
        "qf_graph_begin": (i32, [vp]),
        "qf_graph_end": (vp, [vp]),
        "qf_graph_launch": (i32, [vp, vp]),
        "qf_graph_destroy": (None, [vp]),
        "qfs_create": (vp, [u64, u64]),
        "qfs_destroy": (None, [vp]),
        "qfs_open": (i32, [vp, u32, u32]),
        "qfs_submit": (i32, [vp, i32, i32, vp, u64, vp, u64]),
        "qfs_close": (i32, [vp, i32, u64]),
        "qfs_export": (i32, [vp, i32, ctypes.POINTER(_Layout), u64]),
        "qfs_poll": (i32, [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32), u32, i32]),
        "qfs_stats": (i32, [vp, ctypes.POINTER(ctypes.c_uint64)]),
        "tcf_create": (vp, [u64, i32]),
        "tcf_destroy": (None, [vp]),
        "tcf_insert": (i32, [vp, vp, u64, vp, vp]),
        "tcf_query": (i32, [vp, vp, u64, vp, vp]),
        "tcf_delete": (i32, [vp, vp, u64, vp, vp]),
        "tcf_sync": (i32, [vp, vp]),
        "tcf_info": (i32, [vp, ctypes.POINTER(ctypes.c_uint64), vp]),
        "tcf_export": (i32, [vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _stream(stream) -> int | None:
    if stream is not None:
        return int(stream)
    import torch

    return torch.cuda.current_stream().cuda_stream


def _dev_ptr(t, n: int | None = None, itemsize: int | None = None) -> int:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if itemsize is not None and t.element_size() != itemsize:
        raise ValueError(f"expected {itemsize}-byte elements, got {t.dtype}")
    if n is not None and t.numel() < n:
        raise ValueError("tensor too small")
    return t.data_ptr()


def _check(rc: int, what: str) -> int:
    if rc != QF_OK:
        raise QFError(rc, what)
    return rc


# ---- the C ABI, one wrapper per call ------------------------------------
def qf_create(q: int, r: int) -> int:
    h = lib().qf_create(q, r)
    if not h:
        raise QFError(lib().qf_last_error(), f"qf_create({q}, {r})")
    return h


def qf_destroy(f: int) -> None:
    lib().qf_destroy(f)


def qf_insert_batch(f: int, keys, stream=None) -> int:
    n = keys.numel()
    return lib().qf_insert_batch(f, _dev_ptr(keys, n, 8) if n else None, n, _stream(stream))


def qf_insert_batch_noalloc(f: int, keys, stream=None) -> int:
    n = keys.numel()
    return lib().qf_insert_batch_noalloc(f, _dev_ptr(keys, n, 8) if n else None, n, _stream(stream))


def qf_query_batch(f: int, keys, out, stream=None) -> int:
    n = keys.numel()
    if not n:
        return QF_OK
    return lib().qf_query_batch(f, _dev_ptr(keys, n, 8), n, _dev_ptr(out, n, 1), _stream(stream))


def qf_count_batch(f: int, keys, out, stream=None) -> int:
    n = keys.numel()
    if not n:
        return QF_OK
    return lib().qf_count_batch(f, _dev_ptr(keys, n, 8), n, _dev_ptr(out, n, 8), _stream(stream))


def qf_delete_batch(f: int, keys, not_found=None, stream=None) -> int:
    n = keys.numel()
    nf = _dev_ptr(not_found, 1, 8) if not_found is not None else None
    return lib().qf_delete_batch(f, _dev_ptr(keys, n, 8) if n else None, n, nf, _stream(stream))


def qf_point_insert(f: int, keys, status=None, stream=None) -> int:
    n = keys.numel()
    st = _dev_ptr(status, n, 4) if status is not None and n else None
    return lib().qf_point_insert(f, _dev_ptr(keys, n, 8) if n else None, n, st, _stream(stream))


def qf_point_delete(f: int, keys, status=None, not_found=None, stream=None) -> int:
    n = keys.numel()
    st = _dev_ptr(status, n, 4) if status is not None and n else None
    nf = _dev_ptr(not_found, 1, 8) if not_found is not None else None
    return lib().qf_point_delete(f, _dev_ptr(keys, n, 8) if n else None, n, st, nf, _stream(stream))


def qf_sync(f: int, stream=None) -> int:
    return lib().qf_sync(f, _stream(stream))


def qf_table_bytes(q: int, r: int) -> int:
    return int(lib().qf_table_bytes(q, r))


def qf_last_error() -> int:
    return int(lib().qf_last_error())


def qf_info(f: int) -> dict:
    buf = (ctypes.c_uint64 * 8)()
    _check(lib().qf_info(f, buf), "qf_info")
    keys = ("q", "r", "N", "E", "P", "region_slots", "device_bytes", "batches")
    return dict(zip(keys, (int(v) for v in buf)))


PROF_KINDS = ("hash", "sort_hist", "sort_scan", "sort_scatter", "reduce", "bounds", "merge", "lookup")


def _prof_mask(enable: bool, kinds) -> int:
    """Bit mask of the timed kinds: every kind, or the named ones."""
    if not enable:
        return 0
    if kinds is None:
        return (1 << len(PROF_KINDS)) - 1
    return sum(1 << PROF_KINDS.index(k) for k in set(kinds))


def qf_profile_enable(f: int, enable: bool = True, kinds=None) -> int:
    """Time the launches of the named kinds (default all); enable=False stops."""
    return lib().qf_profile_enable(f, _prof_mask(enable, kinds))


def qf_profile_read(f: int) -> dict:
    """{kind: (milliseconds, launches)} since the last read."""
    ms = (ctypes.c_double * len(PROF_KINDS))()
    n = (ctypes.c_uint64 * len(PROF_KINDS))()
    _check(lib().qf_profile_read(f, ms, n), "qf_profile_read")
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PROF_KINDS)}


def qf_export(f: int, stream=None) -> tuple[int, QFLayout]:
    info = qf_info(f)
    N, P = info["N"], info["P"]
    lay = QFLayout(
        np.zeros(N // 64, np.uint64),
        np.zeros(P // 64, np.uint64),
        np.zeros(P, np.uint16),
        np.zeros(P // 64, np.uint32),
        np.zeros(8, np.uint64),
    )
    c = _Layout()
    c.occ_words = lay.occ_words.ctypes.data
    c.runend_words = lay.runend_words.ctypes.data
    c.slots = lay.slots.ctypes.data
    c.offsets = lay.offsets.ctypes.data
    rc = lib().qf_export(f, ctypes.byref(c), _stream(stream))
    lay.header[:] = np.frombuffer(bytes(c.header), dtype=np.uint64)
    return rc, lay


def qf_import(f: int, lay, stream=None) -> int:
    arrays = [np.ascontiguousarray(lay.occ_words, np.uint64), np.ascontiguousarray(lay.runend_words, np.uint64),
              np.ascontiguousarray(lay.slots, np.uint16), np.ascontiguousarray(lay.offsets, np.uint32)]
    c = _Layout()
    for i, v in enumerate(np.asarray(lay.header, dtype=np.uint64)):
        c.header[i] = int(v)
    c.occ_words, c.runend_words, c.slots, c.offsets = (a.ctypes.data for a in arrays)
    return lib().qf_import(f, ctypes.byref(c), _stream(stream))


class CQF:
    """Owning handle: a counting quotient filter on the current HIP device."""

    def __init__(self, q: int, r: int):
        self.q, self.r = q, r
        self.h = qf_create(q, r)

    def close(self):
        if getattr(self, "h", None):
            qf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, keys, stream=None):
        _check(qf_insert_batch(self.h, keys, stream), "qf_insert_batch")

    def insert_noalloc(self, keys, stream=None):
        """qf_insert_batch_noalloc: the same insert with the library's fixed
        device scratch (batches of at most NOALLOC_MAX_KEYS keys)."""
        _check(qf_insert_batch_noalloc(self.h, keys, stream), "qf_insert_batch_noalloc")

    def delete(self, keys, not_found=None, stream=None):
        _check(qf_delete_batch(self.h, keys, not_found, stream), "qf_delete_batch")

    @classmethod
    def kv(cls, q: int, r: int, vbits: int) -> "CQF":
        """qf_create_kv: a filter that keeps a vbits-bit value with every key."""
        h = lib().qf_create_kv(q, r, vbits)
        if not h:
            raise QFError(lib().qf_last_error(), "qf_create_kv")
        f = cls._own(h, q, r)
        f.vbits = vbits
        return f

    def kv_insert(self, keys, values, stream=None):
        n = keys.numel()
        _check(lib().qf_kv_insert_batch(self.h, _dev_ptr(keys, n, 8) if n else None,
                                        _dev_ptr(values, n, 8) if n else None, n, _stream(stream)),
               "qf_kv_insert_batch")

    def kv_delete(self, keys, values, not_found=None, stream=None):
        n = keys.numel()
        nf = _dev_ptr(not_found, 1, 8) if not_found is not None else None
        _check(lib().qf_kv_delete_batch(self.h, _dev_ptr(keys, n, 8) if n else None,
                                        _dev_ptr(values, n, 8) if n else None, n, nf, _stream(stream)),
               "qf_kv_delete_batch")

    def kv_lookup(self, keys, stream=None):
        """(smallest value per key as int64 bits, 2^64 - 1 when none; number of distinct values)."""
        import torch

        n = keys.numel()
        val = torch.empty(n, dtype=torch.int64, device=keys.device)
        nv = torch.empty(n, dtype=torch.int32, device=keys.device)
        if n:
            _check(lib().qf_kv_lookup_batch(self.h, _dev_ptr(keys, n, 8), n, _dev_ptr(val, n, 8),
                                            _dev_ptr(nv, n, 4), _stream(stream)), "qf_kv_lookup_batch")
        return val, nv

    def point_insert(self, keys, status=None, stream=None):
        """qf_point_insert: one lane per key, in place, each key on its own
        (status: optional int32 device tensor, one code per key)."""
        _check(qf_point_insert(self.h, keys, status, stream), "qf_point_insert")

    def point_delete(self, keys, status=None, not_found=None, stream=None):
        _check(qf_point_delete(self.h, keys, status, not_found, stream), "qf_point_delete")

    def query(self, keys, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        _check(qf_query_batch(self.h, keys, out, stream), "qf_query_batch")
        return out

    def count(self, keys, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
        _check(qf_count_batch(self.h, keys, out, stream), "qf_count_batch")
        return out

    def sync(self, stream=None) -> int:
        return qf_sync(self.h, stream)

    def export(self, stream=None) -> tuple[int, QFLayout]:
        return qf_export(self.h, stream)

    def load(self, lay, stream=None):
        _check(qf_import(self.h, lay, stream), "qf_import")

    def info(self) -> dict:
        return qf_info(self.h)

    @classmethod
    def _own(cls, h: int, q: int, r: int) -> "CQF":
        f = cls.__new__(cls)
        f.q, f.r, f.h = q, r, h
        return f

    def stats(self, stream=None) -> dict:
        """qf_stats: used slots, distinct fingerprints, total count."""
        out = (ctypes.c_uint64 * 3)()
        _check(lib().qf_stats(self.h, out, _stream(stream)), "qf_stats")
        return {"used": int(out[0]), "distinct": int(out[1]), "total": int(out[2])}

    def enumerate(self, stream=None):
        """qf_enumerate: the stored multiset as (fingerprints, counts), two int64
        device tensors holding uint64 values, sorted by fingerprint."""
        import torch

        n = ctypes.c_uint64(0)
        _check(lib().qf_enumerate(self.h, None, None, 0, ctypes.byref(n), _stream(stream)), "qf_enumerate")
        m = int(n.value)
        fp = torch.empty(max(m, 1), dtype=torch.int64, device="cuda")
        cnt = torch.empty(max(m, 1), dtype=torch.int64, device="cuda")
        if m:
            _check(lib().qf_enumerate(self.h, fp.data_ptr(), cnt.data_ptr(), m, ctypes.byref(n), _stream(stream)),
                   "qf_enumerate")
        return fp[:m], cnt[:m]

    def merge_from(self, src: "CQF", subtract: bool = False, not_found=None, stream=None):
        """qf_merge_into(self, src): multiset union (or saturating difference)."""
        nf = None if not_found is None else _dev_ptr(not_found, 1, 8)
        _check(lib().qf_merge_into(self.h, src.h, 1 if subtract else 0, nf, _stream(stream)), "qf_merge_into")

    def resize(self, q: int, r: int, stream=None) -> "CQF":
        """qf_resize: a new filter (q, r), q + r unchanged, with the same multiset."""
        h = lib().qf_resize(self.h, q, r, _stream(stream))
        if not h:
            raise QFError(lib().qf_last_error(), f"qf_resize({q}, {r})")
        f = CQF._own(h, q, r)
        f.vbits = getattr(self, "vbits", 0)
        return f

    def reserve(self, n: int, stream=None):
        _check(lib().qf_reserve(self.h, n, _stream(stream)), "qf_reserve")

    def tune(self, **fields):
        """Launch parameters (qf_tuning_t fields; omitted ones take their defaults)."""
        t = _tuning(fields)
        _check(lib().qf_tune(self.h, ctypes.byref(t)), "qf_tune")

    def tuning(self) -> dict:
        t = _Tuning()
        _check(lib().qf_get_tuning(self.h, ctypes.byref(t)), "qf_get_tuning")
        return _tuning_dict(t)


# ---- filter sets ----------------------------------------------------------
def qf_set_create(filters) -> int:
    hs = (ctypes.c_void_p * len(filters))(*[int(f) for f in filters])
    h = lib().qf_set_create(hs, len(filters))
    if not h:
        raise QFError(lib().qf_last_error(), f"qf_set_create({len(filters)} filters)")
    return h


def qf_set_destroy(s: int) -> None:
    lib().qf_set_destroy(s)


def qf_set_insert_batch(s: int, fid, keys, stream=None) -> int:
    n = keys.numel()
    if not n:
        return QF_OK
    return lib().qf_set_insert_batch(s, _dev_ptr(fid, n, 4), _dev_ptr(keys, n, 8), n, _stream(stream))


def qf_set_delete_batch(s: int, fid, keys, not_found=None, stream=None) -> int:
    n = keys.numel()
    if not n:
        return QF_OK
    nf = _dev_ptr(not_found, None, 8) if not_found is not None else None
    return lib().qf_set_delete_batch(s, _dev_ptr(fid, n, 4), _dev_ptr(keys, n, 8), n, nf, _stream(stream))


def qf_set_query_batch(s: int, fid, keys, out, stream=None) -> int:
    n = keys.numel()
    if not n:
        return QF_OK
    return lib().qf_set_query_batch(s, _dev_ptr(fid, n, 4), _dev_ptr(keys, n, 8), n, _dev_ptr(out, n, 1),
                                    _stream(stream))


def qf_set_count_batch(s: int, fid, keys, out, stream=None) -> int:
    n = keys.numel()
    if not n:
        return QF_OK
    return lib().qf_set_count_batch(s, _dev_ptr(fid, n, 4), _dev_ptr(keys, n, 8), n, _dev_ptr(out, n, 8),
                                    _stream(stream))


def qf_set_sync(s: int, stream=None) -> int:
    return lib().qf_set_sync(s, _stream(stream))


def qf_set_info(s: int) -> dict:
    buf = (ctypes.c_uint64 * 8)()
    _check(lib().qf_set_info(s, buf), "qf_set_info")
    keys = ("nf", "r", "regions", "region_log2_max", "device_bytes", "batches", "key_bits", "_")
    return dict(zip(keys, (int(v) for v in buf)))


def qf_set_profile_enable(s: int, enable: bool = True, kinds=None) -> int:
    return lib().qf_set_profile_enable(s, _prof_mask(enable, kinds))


def qf_set_profile_read(s: int) -> dict:
    ms = (ctypes.c_double * len(PROF_KINDS))()
    n = (ctypes.c_uint64 * len(PROF_KINDS))()
    _check(lib().qf_set_profile_read(s, ms, n), "qf_set_profile_read")
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PROF_KINDS)}


class CQFSet:
    """A set of CQF filters (same r) updated and queried by one pipeline of launches.
    Keys are tagged with int32 filter indices into `filters`; the filters must outlive the set."""

    def __init__(self, filters):
        self.filters = list(filters)
        self.h = qf_set_create([f.h for f in self.filters])

    def close(self):
        if getattr(self, "h", None):
            qf_set_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, fid, keys, stream=None, active=None):
        """active: optional ascending list of the filter indexes the batch touches (only they are merged)."""
        if active is None:
            _check(qf_set_insert_batch(self.h, fid, keys, stream), "qf_set_insert_batch")
            return
        n = keys.numel()
        act = (ctypes.c_uint32 * max(len(active), 1))(*active)
        _check(lib().qf_set_insert_some(self.h, act, len(active), _dev_ptr(fid, n, 4) if n else None,
                                        _dev_ptr(keys, n, 8) if n else None, n, _stream(stream)),
               "qf_set_insert_some")

    def delete(self, fid, keys, not_found=None, stream=None, active=None):
        if active is None:
            _check(qf_set_delete_batch(self.h, fid, keys, not_found, stream), "qf_set_delete_batch")
            return
        n = keys.numel()
        act = (ctypes.c_uint32 * max(len(active), 1))(*active)
        nf = _dev_ptr(not_found, None, 8) if not_found is not None else None
        _check(lib().qf_set_delete_some(self.h, act, len(active), _dev_ptr(fid, n, 4) if n else None,
                                        _dev_ptr(keys, n, 8) if n else None, n, nf, _stream(stream)),
               "qf_set_delete_some")

    def query(self, fid, keys, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        _check(qf_set_query_batch(self.h, fid, keys, out, stream), "qf_set_query_batch")
        return out

    def count(self, fid, keys, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty(keys.numel(), dtype=torch.int64, device=keys.device)
        _check(qf_set_count_batch(self.h, fid, keys, out, stream), "qf_set_count_batch")
        return out

    def sync(self, stream=None) -> int:
        return qf_set_sync(self.h, stream)

    def errors(self, stream=None) -> tuple[int, np.ndarray]:
        """Waits for `stream`; (number of filters with a deferred error, each filter's code), cleared."""
        codes = np.zeros(len(self.filters), dtype=np.int32)
        n = lib().qf_set_errors(self.h, codes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream(stream))
        return int(n), codes

    def info(self) -> dict:
        return qf_set_info(self.h)

    def reserve(self, n: int, stream=None):
        _check(lib().qf_set_reserve(self.h, n, _stream(stream)), "qf_set_reserve")

    def tune(self, **fields):
        t = _tuning(fields)
        _check(lib().qf_set_tune(self.h, ctypes.byref(t)), "qf_set_tune")

    def tuning(self) -> dict:
        t = _Tuning()
        _check(lib().qf_set_get_tuning(self.h, ctypes.byref(t)), "qf_set_get_tuning")
        return _tuning_dict(t)


def autotune_set(qs, r: int, load: float, n_query: int) -> tuple[dict, tuple[float, float]]:
    """qf_autotune_set: the launch parameters the library's autotuner picks for a set of filters with
    quotient bits `qs`, filled to `load` by one insert batch and queried in batches of n_query keys;
    also the sample's insert and query milliseconds under them."""
    arr = (ctypes.c_uint32 * len(qs))(*[int(q) for q in qs])
    t = _Tuning()
    ms = (ctypes.c_double * 2)()
    _check(lib().qf_autotune_set(arr, len(qs), r, float(load), int(n_query), ctypes.byref(t), ms),
           "qf_autotune_set")
    return _tuning_dict(t), (ms[0], ms[1])


class Graph:
    """Batch calls captured on a stream (qf_graph_begin / qf_graph_end) and replayed with launch().

        g = Graph(stream)            # starts capturing `stream` (a torch.cuda.Stream)
        with g: ...batch calls on stream...
        g.launch()                   # replay on the same stream
    """

    def __init__(self, stream):
        self.stream = stream
        self.h = None

    def __enter__(self):
        _check(lib().qf_graph_begin(int(self.stream.cuda_stream)), "qf_graph_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        h = lib().qf_graph_end(int(self.stream.cuda_stream))
        if exc_type is not None:
            if h:
                lib().qf_graph_destroy(h)
            return False
        if not h:
            raise QFError(lib().qf_last_error(), "qf_graph_end")
        self.h = h
        return False

    def launch(self, stream=None):
        s = self.stream if stream is None else stream
        _check(lib().qf_graph_launch(self.h, int(s.cuda_stream)), "qf_graph_launch")

    def close(self):
        if getattr(self, "h", None):
            lib().qf_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving --------------------------------------------------------------
QFS_INSERT, QFS_DELETE, QFS_QUERY, QFS_COUNT = 0, 1, 2, 3


class ServedExport:
    """Host arrays a served filter's table is copied into (Server.export)."""

    def __init__(self, lay: QFLayout):
        self.lay = lay
        self.c = _Layout()

    def layout(self) -> QFLayout:
        self.lay.header[:] = np.frombuffer(bytes(self.c.header), dtype=np.uint64)
        return self.lay


class Server:
    """Device-resident filters answering host requests with continuous batching (qfs_* calls).
    Keys are host numpy uint64 arrays; outputs are host numpy arrays kept alive until completion."""

    def __init__(self, budget_bytes: int, max_round_keys: int = 1 << 22):
        self.h = lib().qfs_create(budget_bytes, max_round_keys)
        if not self.h:
            raise QFError(QF_ERR_OOM, "qfs_create")
        self._live = {}  # tag -> (keys, out) kept alive until polled

    def close(self):
        if getattr(self, "h", None):
            lib().qfs_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open(self, q: int, r: int) -> int:
        rc = lib().qfs_open(self.h, q, r)
        if rc < 0:
            raise QFError(rc, f"qfs_open({q}, {r})")
        return rc

    def submit(self, op: int, fid: int, keys: np.ndarray, tag: int) -> np.ndarray | None:
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        n = len(keys)
        out = None
        if op == QFS_QUERY:
            out = np.zeros(n, np.uint8)
        elif op == QFS_COUNT:
            out = np.zeros(n, np.uint64)
        rc = lib().qfs_submit(self.h, op, fid, keys.ctypes.data if n else None, n,
                              out.ctypes.data if out is not None and n else None, tag)
        _check(rc, "qfs_submit")
        self._live[tag] = (keys, out)
        return out

    def close_filter(self, fid: int, tag: int):
        _check(lib().qfs_close(self.h, fid, tag), "qfs_close")
        self._live[tag] = (None, None)

    def export(self, fid: int, q: int, r: int, tag: int) -> "ServedExport":
        """qfs_export: the filter's table after its requests submitted so far.  The returned object's
        layout() is valid once the completion with `tag` has been polled (status QF_OK)."""
        nblocks = qf_table_bytes(q, r) // (128 if r == 8 else 160)
        P = nblocks * 64
        ex = ServedExport(QFLayout(np.zeros((1 << q) // 64, np.uint64), np.zeros(P // 64, np.uint64),
                                   np.zeros(P, np.uint16), np.zeros(P // 64, np.uint32), np.zeros(8, np.uint64)))
        c = ex.c
        c.occ_words = ex.lay.occ_words.ctypes.data
        c.runend_words = ex.lay.runend_words.ctypes.data
        c.slots = ex.lay.slots.ctypes.data
        c.offsets = ex.lay.offsets.ctypes.data
        _check(lib().qfs_export(self.h, fid, ctypes.byref(c), tag), "qfs_export")
        self._live[tag] = (ex, None)
        return ex

    def poll(self, max_n: int = 4096, wait_us: int = 1000) -> list[tuple[int, int]]:
        tags = (ctypes.c_uint64 * max_n)()
        st = (ctypes.c_int32 * max_n)()
        k = lib().qfs_poll(self.h, tags, st, max_n, wait_us)
        if k < 0:
            raise QFError(k, "qfs_poll")
        res = [(int(tags[i]), int(st[i])) for i in range(k)]
        for t, _ in res:
            self._live.pop(t, None)
        return res

    def stats(self) -> dict:
        buf = (ctypes.c_uint64 * 15)()
        _check(lib().qfs_stats(self.h, buf), "qfs_stats")
        keys = ("rounds", "requests", "keys", "open", "pending", "bytes_used", "budget", "waiting",
                "updates_in_place", "updates_bulk", "ns_form", "ns_launch", "ns_wait", "ns_complete", "ns_stage")
        return dict(zip(keys, (int(v) for v in buf)))
