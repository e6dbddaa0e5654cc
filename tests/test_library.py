"""The C-ABI library loads and exports every call include/qf.h declares (no GPU).

Only symbol lookups and the argument checks that return before touching the
device are exercised here; every compute call needs a GPU (tests marked gpu).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import pytest

from paper_2212_09005_amd import qf

pytestmark = pytest.mark.skipif(not os.path.exists(qf.LIB_PATH), reason="libqf.so not built")


def test_header_declares_the_api():
    names = qf.declared_functions()
    for want in ("qf_create", "qf_insert_batch", "qf_query_batch", "qf_count_batch", "qf_delete_batch",
                 "qf_destroy", "qf_sync", "qf_export", "qf_import", "qf_last_error", "qf_table_bytes",
                 "qf_info", "qf_profile_enable", "qf_profile_read"):
        assert want in names


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(qf.LIB_PATH)
    for name in qf.declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", qf.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(qf.declared_functions()) <= exported


def test_library_is_built_for_gfx950():
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", qf.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_argument_errors_return_before_the_device():
    L = qf.lib()
    assert L.qf_create(5, 8) is None and L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qf_create(12, 7) is None and L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qf_create(32, 8) is None and L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qf_insert_batch(None, None, 5, None) == qf.QF_ERR_ARG
    assert L.qf_query_batch(None, None, 5, None, None) == qf.QF_ERR_ARG
    assert L.qf_count_batch(None, None, 5, None, None) == qf.QF_ERR_ARG
    assert L.qf_delete_batch(None, None, 5, None, None) == qf.QF_ERR_ARG
    assert L.qf_sync(None, None) == qf.QF_ERR_ARG
    # tuning, autotuning and capture calls check their arguments first too
    assert L.qf_tune(None, None) == qf.QF_ERR_ARG
    assert L.qf_set_tune(None, None) == qf.QF_ERR_ARG
    assert L.qf_get_tuning(None, None) == qf.QF_ERR_ARG
    t = qf._Tuning()
    qs = (ctypes.c_uint32 * 2)(10, 12)
    assert L.qf_autotune_set(None, 2, 8, 0.85, 1000, ctypes.byref(t), None) == qf.QF_ERR_ARG
    assert L.qf_autotune_set(qs, 2, 7, 0.85, 1000, ctypes.byref(t), None) == qf.QF_ERR_ARG
    assert L.qf_autotune_set(qs, 2, 8, 1.5, 1000, ctypes.byref(t), None) == qf.QF_ERR_ARG
    bad_q = (ctypes.c_uint32 * 1)(40)
    assert L.qf_autotune_set(bad_q, 1, 8, 0.5, 1000, ctypes.byref(t), None) == qf.QF_ERR_ARG
    assert L.qf_graph_begin(None) == qf.QF_ERR_ARG
    assert L.qf_graph_end(None) is None and L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qf_graph_launch(None, None) == qf.QF_ERR_ARG
    L.qf_graph_destroy(None)
    L.qf_destroy(None)


def test_table_bytes():
    # 128-byte blocks (r = 8) or 160-byte blocks (r = 16), offset inside
    assert qf.qf_table_bytes(16, 8) == (65536 + 2560) // 64 * 128
    assert qf.qf_table_bytes(28, 8) == ((1 << 28) + 163840) // 64 * 128
    assert qf.qf_table_bytes(30, 16) == ((1 << 30) + 327680) // 64 * 160
    assert qf.qf_table_bytes(5, 8) == 0
