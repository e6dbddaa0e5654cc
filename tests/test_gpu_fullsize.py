"""Parity at the benchmark's full size (2^28 quotients, r = 8, load 0.9).

The GPU table is filled with the benchmark's own key stream and batch size
(the launch configuration bench.py times), exported, and compared bit for bit
with the canonical table the definition oracle (oracle/brute.py) builds from
the same multiset; then one benchmark step (insert a batch, query, count,
delete it) is checked the same way.  The host side needs ~25 GB of memory and
about a minute per table.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

from oracle import brute
from paper_2212_09005_amd.workloads import C2

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]

U64 = np.uint64


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def compare(lay, ref, what):
    for name in ("occ_words", "runend_words", "slots", "offsets", "header"):
        a = np.asarray(getattr(lay, name)).astype(U64)
        b = np.asarray(getattr(ref, name)).astype(U64)
        bad = np.nonzero(a != b)[0]
        assert len(bad) == 0, f"{what}: {name} differs in {len(bad)} places, first {int(bad[0])}"


def test_full_size_load_sweep_table_and_step():
    from paper_2212_09005_amd import qf

    w = C2
    note(f"full size q={w.q} r={w.r} load={w.load} batch={w.batch}")
    t0 = time.time()
    fill = w.fill_keys()
    f = qf.CQF(w.q, w.r)
    d = torch.empty(w.batch, dtype=torch.int64, device="cuda")
    for s in range(0, len(fill), w.batch):
        part = fill[s : s + w.batch]
        d[: len(part)].copy_(torch.from_numpy(part.view(np.int64)))
        f.insert(d[: len(part)])
    assert f.sync() == 0
    rc, lay = f.export()
    assert rc == 0
    note(f"gpu fill + export {time.time() - t0:.0f}s")
    ms0 = brute.multiset(brute.fingerprints(fill, w.q, w.r))
    compare(lay, brute.layout(ms0[0], ms0[1], w.q, w.r), "filled table")
    del lay
    note(f"filled table bit-exact ({time.time() - t0:.0f}s)")

    # one benchmark step
    ins = w.insert_keys(0)
    qk = w.query_keys(0, fill)
    di = torch.from_numpy(ins.view(np.int64)).cuda()
    dq = torch.from_numpy(qk.view(np.int64)).cuda()
    f.insert(di)
    got_q = f.query(dq).cpu().numpy()
    got_c = f.count(dq).cpu().numpy().view(U64)
    rc, lay1 = f.export()
    assert rc == 0
    ms1 = brute.merge_multisets(ms0, brute.multiset(brute.fingerprints(ins, w.q, w.r)))
    want_c = brute.counts_of(ms1[0], ms1[1], brute.fingerprints(qk, w.q, w.r))
    assert np.array_equal(got_c, want_c)
    assert np.array_equal(got_q, (want_c > 0).astype(np.uint8))
    compare(lay1, brute.layout(ms1[0], ms1[1], w.q, w.r), "after the step's insert")
    del lay1
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    f.delete(di, nf)
    rc, lay2 = f.export()
    assert rc == 0 and int(nf.item()) == 0
    compare(lay2, brute.layout(ms0[0], ms0[1], w.q, w.r), "after the step's delete")
    note(f"step bit-exact ({time.time() - t0:.0f}s)")
    f.close()
