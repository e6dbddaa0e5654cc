"""Python binding of the two-choice filter calls of include/tcf.h.

Argument marshalling only: every operation runs in the HIP library
(libqf.so); there is no fallback.  Keys, statuses and outputs are device
tensors (torch, on the filter's GPU).
"""
from __future__ import annotations

import ctypes

import numpy as np

from .qf import QF_OK, QFError, _check, _dev_ptr, _stream, lib

TCF_POINT = 0
TCF_BULK = 1


class TCF:
    """A two-choice filter of `nblocks` blocks: kind TCF_POINT (16 tags per
    block, one lane per key, lock-free) or TCF_BULK (128 sorted tags per
    block, batches sorted and merged)."""

    def __init__(self, nblocks: int, kind: int = TCF_POINT):
        h = lib().tcf_create(nblocks, kind)
        if not h:
            raise QFError(lib().qf_last_error(), "tcf_create")
        self.h = h
        self.kind = kind
        info = self.info()
        self.nblocks, self.B, self.backing_entries = info["nblocks"], info["tags_per_block"], info["backing_entries"]

    def close(self):
        if self.h:
            lib().tcf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, keys, status=None, stream=None):
        n = keys.numel()
        st = _dev_ptr(status, n, 4) if status is not None and n else None
        _check(lib().tcf_insert(self.h, _dev_ptr(keys, n, 8) if n else None, n, st, _stream(stream)), "tcf_insert")

    def query(self, keys, out=None, stream=None):
        import torch

        n = keys.numel()
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=keys.device)
        if n:
            _check(lib().tcf_query(self.h, _dev_ptr(keys, n, 8), n, _dev_ptr(out, n, 1), _stream(stream)),
                   "tcf_query")
        return out

    def delete(self, keys, not_found=None, stream=None):
        n = keys.numel()
        nf = _dev_ptr(not_found, 1, 8) if not_found is not None else None
        _check(lib().tcf_delete(self.h, _dev_ptr(keys, n, 8) if n else None, n, nf, _stream(stream)), "tcf_delete")

    def sync(self, stream=None) -> int:
        return lib().tcf_sync(self.h, _stream(stream))

    def info(self, stream=None) -> dict:
        out = (ctypes.c_uint64 * 7)()
        _check(lib().tcf_info(self.h, out, _stream(stream)), "tcf_info")
        keys = ("kind", "nblocks", "tags_per_block", "backing_entries", "backing_used", "held", "device_bytes")
        return dict(zip(keys, (int(v) for v in out)))

    def export(self, stream=None):
        """(slots as a (nblocks, B) uint16 array, backing table as uint64)."""
        slots = np.zeros((self.nblocks, self.B), dtype=np.uint16)
        bk = np.zeros(self.backing_entries, dtype=np.uint64)
        rc = lib().tcf_export(self.h, slots.ctypes.data, bk.ctypes.data, _stream(stream))
        if rc != QF_OK:
            raise QFError(rc, "tcf_export")
        return slots, bk
