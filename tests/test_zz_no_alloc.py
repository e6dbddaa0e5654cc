"""qf_insert_batch_noalloc (batch scratch in the library's fixed device array)
gives the same table as qf_insert_batch, over two calls in a row on two
filters, the second call with a smaller batch, and refuses a batch above its
limit without touching the filter."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_2212_09005_amd import inputs, qf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("occ_words", "runend_words", "slots", "offsets", "header")


def _same(a, b, what):
    for name in FIELDS:
        x = np.asarray(getattr(a, name)).astype(np.uint64)
        y = np.asarray(getattr(b, name)).astype(np.uint64)
        assert np.array_equal(x, y), f"{what}: {name} differs"


@pytest.mark.parametrize("q,r", [(20, 8), (20, 16)])
def test_noalloc_insert_equals_insert(q, r):
    print(f"[case] noalloc insert vs insert q={q} r={r}", flush=True)
    lib = qf.lib()
    a, b = qf.CQF(q, r), qf.CQF(q, r)
    # first call: the largest batch the static scratch takes; second: smaller
    # (the radix path), third: a small batch (the one-work-group path)
    sizes = [qf.NOALLOC_MAX_KEYS, 150_000, 3_000]
    for i, n in enumerate(sizes):
        keys = inputs.uniform_keys(900 + i, n)
        keys[: n // 10] = keys[n // 10 : 2 * (n // 10)]  # duplicates are counted
        d = torch.from_numpy(keys.view(np.int64)).cuda()
        a.insert(d)
        b.insert_noalloc(d)
        assert a.sync() == 0 and b.sync() == 0
        ra, la = a.export()
        rb, lb = b.export()
        assert ra == 0 and rb == 0
        _same(la, lb, f"after call {i + 1} ({n} keys)")
    # above the limit: refused at once, the filter is unchanged
    big = torch.zeros(qf.NOALLOC_MAX_KEYS + 1, dtype=torch.int64, device="cuda")
    rc = lib.qf_insert_batch_noalloc(b.h, ctypes.c_void_p(big.data_ptr()), big.numel(),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == qf.QF_ERR_LIMIT and lib.qf_last_error() == qf.QF_ERR_LIMIT
    assert b.sync() == 0
    _, lb2 = b.export()
    _same(la, lb2, "after the refused batch")
    a.close()
    b.close()
