"""GPU tests of the serving loop (qfs_*): requests submitted without waiting
are batched into rounds with others, yet every answer must equal the answer of
executing that filter's requests one at a time in submission order (the
sequential oracle replays them), and filters beyond the HBM budget wait for
admission without blocking the others.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

from oracle import oqf
from paper_2212_09005_amd import inputs

pytestmark = pytest.mark.gpu

U64 = np.uint64


def _qf():
    from paper_2212_09005_amd import qf

    return qf


def note(msg: str):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def drain(srv, want: int, timeout_s: float = 60.0):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < want:
        assert time.time() < t_end, f"only {len(got)} of {want} completions"
        for tag, st in srv.poll(4096, 20000):
            got[tag] = st
    return got


def test_serving_mix_equals_sequential_replay():
    qf = _qf()
    note("serving: mixed requests on 6 filters vs sequential replay")
    rng = np.random.Generator(np.random.PCG64(17))
    shapes = [(10, 8), (12, 8), (11, 16), (13, 16), (9, 8), (14, 8)]
    srv = qf.Server(8 << 30, max_round_keys=1 << 16)
    ids = [srv.open(q, r) for q, r in shapes]
    oracles = [oqf.OracleQF(q, r) for q, r in shapes]
    present = [np.zeros(0, U64) for _ in shapes]
    reqs = []  # (tag, op, filter, keys, out)
    tag = 0
    for i in range(600):
        f = int(rng.integers(0, len(shapes)))
        q, r = shapes[f]
        u = rng.random()
        n = int(2 ** rng.uniform(0, 9))
        if u < 0.25 or len(present[f]) == 0:
            op = qf.QFS_INSERT
            room = int(0.8 * (1 << q)) - len(present[f])
            n = max(0, min(n, room))
            keys = inputs.uniform_keys(10_000 + i, n)
            present[f] = np.concatenate([present[f], keys])
        elif u < 0.3:
            op = qf.QFS_DELETE
            keys = present[f][rng.integers(0, len(present[f]), n)]
        else:
            op = qf.QFS_QUERY if u < 0.65 else qf.QFS_COUNT
            keys = np.concatenate([present[f][rng.integers(0, len(present[f]), n // 2 + 1)],
                                   inputs.absent_keys(20_000 + i, n // 2)])
        out = srv.submit(op, ids[f], keys, tag)
        reqs.append((tag, op, f, keys, out))
        tag += 1
    got = drain(srv, len(reqs))
    assert all(st == 0 for st in got.values()), {t: s for t, s in got.items() if s}
    # replay one request at a time, in submission order, per filter
    for t, op, f, keys, out in reqs:
        o = oracles[f]
        if op == qf.QFS_INSERT:
            if len(keys):
                assert o.insert(keys) == 0
        elif op == qf.QFS_DELETE:
            if len(keys):
                assert o.delete(keys)[0] == 0
        else:
            want = o.count(keys) if len(keys) else np.zeros(0, U64)
            if op == qf.QFS_COUNT:
                assert np.array_equal(out, want), f"request {t}: counts differ"
            else:
                assert np.array_equal(out, (want > 0).astype(np.uint8)), f"request {t}: answers differ"
    st = srv.stats()
    note(f"rounds {st['rounds']} for {st['requests']} requests")
    assert st["rounds"] < len(reqs), "no batching happened"
    # the final tables: every key ever inserted, counted through the server
    for f in range(len(shapes)):
        probe = present[f][:4000]
        out = srv.submit(qf.QFS_COUNT, ids[f], probe, 100_000 + f)
        drain(srv, 1)
        assert np.array_equal(out, oracles[f].count(probe))
    srv.close()


def test_serving_admission_by_budget():
    qf = _qf()
    note("serving: third filter waits for budget")
    # what one q=16 filter costs in the server's own accounting
    probe = qf.Server(1 << 34, max_round_keys=1 << 12)
    used0 = probe.stats()["bytes_used"]
    probe.open(16, 8)
    time.sleep(0.2)
    cost = probe.stats()["bytes_used"] - used0
    probe.close()
    assert cost > 0
    srv = qf.Server(used0 + int(2.5 * cost), max_round_keys=1 << 12)
    a, b, c = srv.open(16, 8), srv.open(16, 8), srv.open(16, 8)
    keys = inputs.uniform_keys(5, 3000)
    srv.submit(qf.QFS_INSERT, a, keys, 1)
    srv.submit(qf.QFS_INSERT, c, keys[:100], 2)  # waits: c is not admitted yet
    got = drain(srv, 1)
    assert 1 in got and 2 not in got
    time.sleep(0.2)
    assert srv.stats()["pending"] == 1
    assert not srv.poll(16, 1000)
    srv.close_filter(b, 3)  # frees room: c is admitted, its insert runs
    got = drain(srv, 2)
    assert got.get(2) == 0 and got.get(3) == 0
    out = srv.submit(qf.QFS_COUNT, c, keys[:200], 4)
    drain(srv, 1)
    o = oqf.OracleQF(16, 8)
    assert o.insert(keys[:100]) == 0
    assert np.array_equal(out, o.count(keys[:200]))
    assert srv.stats()["pending"] == 0
    srv.close()
    s2 = qf.Server(1 << 20, max_round_keys=1 << 10)
    with pytest.raises(qf.QFError):
        s2.open(28, 8)
    s2.close()
