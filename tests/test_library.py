"""The C-ABI library loads and exports every call include/qf.h declares (no GPU).

Only symbol lookups and the argument checks that return before touching the
device are exercised here; every compute call needs a GPU (tests marked gpu).
"""
from __future__ import annotations

import ctypes
import os
import struct
import subprocess
import sys

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


def _offload_targets(path):
    """Target ids of the device code bundled in a HIP library: clang's offload
    bundle starts with a 24-byte magic, then a u64 entry count, then per entry
    u64 offset, u64 size, u64 id length and the id text."""
    data = open(path, "rb").read()
    at = data.find(b"__CLANG_OFFLOAD_BUNDLE__")
    assert at >= 0, "no offload bundle in the library"
    o = at + 24
    (n,) = struct.unpack_from("<Q", data, o)
    o += 8
    ids = []
    for _ in range(n):
        _off, size, idlen = struct.unpack_from("<QQQ", data, o)
        o += 24
        ids.append((data[o:o + idlen].decode(), size))
        o += idlen
    return ids


def test_library_is_built_for_gfx950():
    ids = _offload_targets(qf.LIB_PATH)
    device = [(i, size) for i, size in ids if i.startswith("hip")]
    # one device code object, for gfx950 only, and not empty
    assert len(device) == 1 and device[0][0].endswith("--gfx950") and device[0][1] > 0, ids


def test_argument_errors_return_before_the_device():
    L = qf.lib()
    assert L.qf_create(5, 8) is None and L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qf_create(12, 7) is None and L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qf_create(32, 8) is None and L.qf_last_error() == qf.QF_ERR_ARG
    # q = 31 is refused too: the CPU checker builds tables up to q = 30 only
    assert L.qf_create(31, 8) is None and L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qfs_open(None, 12, 8) == qf.QF_ERR_ARG
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


def test_set_create_refuses_null_and_repeated_handles():
    # both are found by comparing the handles, before any handle is read, so
    # stand-in addresses (never dereferenced) exercise the check without a GPU
    L = qf.lib()
    buf = (ctypes.c_uint8 * 64)()
    a = ctypes.addressof(buf)
    for hs in ([a, a], [a, a + 16, a], [a + 16, 0], [0]):
        arr = (ctypes.c_void_p * len(hs))(*hs)
        assert L.qf_set_create(arr, len(hs)) is None
        assert L.qf_last_error() == qf.QF_ERR_ARG
    assert L.qf_set_create(None, 2) is None and L.qf_last_error() == qf.QF_ERR_ARG


def test_table_bytes():
    # 128-byte blocks (r = 8) or 160-byte blocks (r = 16), offset inside
    assert qf.qf_table_bytes(16, 8) == (65536 + 2560) // 64 * 128
    assert qf.qf_table_bytes(28, 8) == ((1 << 28) + 163840) // 64 * 128
    assert qf.qf_table_bytes(30, 16) == ((1 << 30) + 327680) // 64 * 160
    assert qf.qf_table_bytes(5, 8) == 0
    assert qf.qf_table_bytes(31, 8) == 0


def _run_py(code):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=root)


def test_missing_library_fails_loudly():
    # with the library path pointing nowhere, the first call raises: there is
    # no other implementation to fall back to
    out = _run_py(
        "from paper_2212_09005_amd import qf\n"
        "qf.LIB_PATH = '/nonexistent/libqf.so'\n"
        "qf._lib = None\n"
        "try:\n"
        "    qf.lib()\n"
        "except ImportError as e:\n"
        "    print('raised:', e)\n"
    )
    assert out.returncode == 0, out.stderr
    assert "raised:" in out.stdout and "no fallback" in out.stdout


def test_package_does_not_load_the_oracle():
    out = _run_py(
        "import sys\n"
        "import paper_2212_09005_amd\n"
        "from paper_2212_09005_amd import qf, inputs, workloads\n"
        "print(sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')))\n"
    )
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "[]"
