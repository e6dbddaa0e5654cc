"""ctypes wrapper of the plain sequential CPU counting quotient filter (oqf.c).

TEST INFRASTRUCTURE ONLY: the oracle the GPU library is checked against.  Only
tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import it.
It shares no code with the HIP library.

The filter it wraps follows the paper's CQF description (Sec. 5.1: quotient /
remainder split, runs, clusters, shifting; Sec. 5.3: remainders sorted within
a run; Sec. 5.4: aggregated counts; Sec. 6.4: deletes shift left).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboqf.so")

OQF_OK = 0
OQF_ERR_ARG = -1
OQF_ERR_FULL = -2
OQF_ERR_OOM = -3
OQF_ERR_COUNT_OVERFLOW = -5


def build(force: bool = False) -> str:
    """Compile oqf.c into liboqf.so next to it (plain gcc, no GPU code)."""
    import subprocess

    src = os.path.join(_HERE, "oqf.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.oqf_fin64.restype = u64
        L.oqf_fin64.argtypes = [u64]
        L.oqf_create.restype = vp
        L.oqf_create.argtypes = [u32, u32]
        L.oqf_destroy.argtypes = [vp]
        L.oqf_num_slots.restype = u64
        L.oqf_num_slots.argtypes = [vp]
        L.oqf_num_extra.restype = u64
        L.oqf_num_extra.argtypes = [vp]
        L.oqf_extra_slots.restype = u64
        L.oqf_extra_slots.argtypes = [u32]
        L.oqf_fingerprint.restype = u64
        L.oqf_fingerprint.argtypes = [vp, u64]
        L.oqf_insert_batch.restype = ctypes.c_int
        L.oqf_insert_batch.argtypes = [vp, vp, u64]
        L.oqf_insert_fp_counts.restype = ctypes.c_int
        L.oqf_insert_fp_counts.argtypes = [vp, vp, vp, u64]
        L.oqf_delete_batch.restype = ctypes.c_int
        L.oqf_delete_batch.argtypes = [vp, vp, u64, vp]
        L.oqf_count_batch.restype = None
        L.oqf_count_batch.argtypes = [vp, vp, u64, vp]
        L.oqf_query_batch.restype = None
        L.oqf_query_batch.argtypes = [vp, vp, u64, vp]
        L.oqf_export.restype = ctypes.c_int
        L.oqf_export.argtypes = [vp, vp, vp, vp, vp, vp]
        L.oqf_import.restype = ctypes.c_int
        L.oqf_import.argtypes = [vp, vp, vp, vp, vp]
        L.oqf_max_cluster.restype = u64
        L.oqf_max_cluster.argtypes = [vp]
        L.oqf_encode_entry.restype = u64
        L.oqf_encode_entry.argtypes = [u32, u64, u64, vp]
        L.oqf_decode_entry.restype = ctypes.c_int
        L.oqf_decode_entry.argtypes = [u32, vp, u64, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Layout:
    """Logical table: the same fields the GPU library's qf_export produces."""

    occ_words: np.ndarray  # uint64[N/64]
    runend_words: np.ndarray  # uint64[P/64]
    slots: np.ndarray  # uint16[P]
    offsets: np.ndarray  # uint32[P/64]
    header: np.ndarray  # uint64[8]: q, r, N, E, P, used, distinct, total

    def equal(self, other: "Layout") -> bool:
        return (
            np.array_equal(self.occ_words, other.occ_words)
            and np.array_equal(self.runend_words, other.runend_words)
            and np.array_equal(self.slots.astype(np.uint16), other.slots.astype(np.uint16))
            and np.array_equal(self.offsets, other.offsets)
            and np.array_equal(self.header, other.header)
        )

    def diff(self, other: "Layout") -> str:
        out = []
        for name in ("occ_words", "runend_words", "slots", "offsets", "header"):
            a = getattr(self, name).astype(np.uint64)
            b = getattr(other, name).astype(np.uint64)
            if a.shape != b.shape:
                out.append(f"{name}: shape {a.shape} vs {b.shape}")
                continue
            bad = np.nonzero(a != b)[0]
            if len(bad):
                i = bad[0]
                out.append(f"{name}: {len(bad)} mismatches, first at {i}: {a[i]:#x} vs {b[i]:#x}")
        return "; ".join(out) if out else "identical"


def fin64(x: int) -> int:
    return int(lib().oqf_fin64(x))


def extra_slots(q: int) -> int:
    return int(lib().oqf_extra_slots(q))


def encode_entry(r: int, x: int, c: int) -> list[int]:
    buf = np.zeros(96, dtype=np.uint16)
    n = lib().oqf_encode_entry(r, x, c, _ptr(buf))
    if n == 0:
        raise ValueError("bad entry")
    return [int(v) for v in buf[:n]]


def decode_entry(r: int, slots) -> tuple[int, int, int]:
    buf = np.asarray(slots, dtype=np.uint16)
    x = ctypes.c_uint64()
    c = ctypes.c_uint64()
    used = ctypes.c_uint64()
    rc = lib().oqf_decode_entry(r, _ptr(buf), len(buf), ctypes.byref(x), ctypes.byref(c), ctypes.byref(used))
    if rc:
        raise ValueError("invalid encoding")
    return int(x.value), int(c.value), int(used.value)


class OracleQF:
    """One plain CPU counting quotient filter with the batch calls of the GPU API."""

    def __init__(self, q: int, r: int):
        self.q, self.r = q, r
        self._h = lib().oqf_create(q, r)
        if not self._h:
            raise ValueError(f"oqf_create({q}, {r}) rejected")
        self.P = int(lib().oqf_num_slots(self._h))
        self.E = int(lib().oqf_num_extra(self._h))
        self.N = 1 << q

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oqf_destroy(h)
            self._h = None

    def fingerprint(self, key: int) -> int:
        return int(lib().oqf_fingerprint(self._h, key))

    def insert(self, keys: np.ndarray) -> int:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        return int(lib().oqf_insert_batch(self._h, _ptr(k), len(k)))

    def insert_fp_counts(self, fps: np.ndarray, counts: np.ndarray) -> int:
        f = np.ascontiguousarray(fps, dtype=np.uint64)
        c = np.ascontiguousarray(counts, dtype=np.uint64)
        return int(lib().oqf_insert_fp_counts(self._h, _ptr(f), _ptr(c), len(f)))

    def delete(self, keys: np.ndarray) -> tuple[int, int]:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        nf = np.zeros(1, dtype=np.uint64)
        rc = int(lib().oqf_delete_batch(self._h, _ptr(k), len(k), _ptr(nf)))
        return rc, int(nf[0])

    def count(self, keys: np.ndarray) -> np.ndarray:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(len(k), dtype=np.uint64)
        lib().oqf_count_batch(self._h, _ptr(k), len(k), _ptr(out))
        return out

    def query(self, keys: np.ndarray) -> np.ndarray:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(len(k), dtype=np.uint8)
        lib().oqf_query_batch(self._h, _ptr(k), len(k), _ptr(out))
        return out

    def export(self) -> Layout:
        occ = np.zeros(self.N // 64, dtype=np.uint64)
        rend = np.zeros(self.P // 64, dtype=np.uint64)
        slots = np.zeros(self.P, dtype=np.uint16)
        offs = np.zeros(self.P // 64, dtype=np.uint32)
        hdr = np.zeros(8, dtype=np.uint64)
        rc = lib().oqf_export(self._h, _ptr(occ), _ptr(rend), _ptr(slots), _ptr(offs), _ptr(hdr))
        if rc:
            raise RuntimeError("oqf_export failed")
        return Layout(occ, rend, slots, offs, hdr)

    def load(self, lay: Layout) -> None:
        """Replace the table by a logical layout (e.g. one brute.layout built)."""
        occ = np.ascontiguousarray(lay.occ_words, dtype=np.uint64)
        rend = np.ascontiguousarray(lay.runend_words, dtype=np.uint64)
        slots = np.ascontiguousarray(lay.slots, dtype=np.uint16)
        hdr = np.ascontiguousarray(lay.header, dtype=np.uint64)
        rc = lib().oqf_import(self._h, _ptr(occ), _ptr(rend), _ptr(slots), _ptr(hdr))
        if rc:
            raise ValueError(f"oqf_import rejected the layout ({rc})")

    def max_cluster(self) -> int:
        return int(lib().oqf_max_cluster(self._h))
