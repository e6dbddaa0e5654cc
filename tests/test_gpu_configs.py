"""Parity at the shapes of the counting, many-filter and serving workloads.

Each test runs the HIP library through its C ABI at the workload's real shape
(the sizes bench.py runs) and compares what it can with the definition oracle
(oracle/brute.py): whole tables bit for bit, and answers element by element.

  * counting with skew: 2^30 quotients, r = 16, 0.9 * 2^30 Zipf(1.1) instances
    over 2^28 values in ONE batch; the table after the insert and after the
    delete of a random quarter of the instances, and exact counts of 2^26 keys;
  * many filters: 4096 filters (2^10..2^20 quotients, r = 8) filled to load
    0.85 by one set batch, then 2^24 queries and counts routed by filter;
    264 filters (24 of every size) compared table by table;
  * serving: 256 filters (2^18..2^26 quotients, r = 8 or 16) at load 0.5 and a
    stream of mixed requests of 1..65,536 keys served with continuous
    batching; every answer equals the same stream run one request at a time,
    and the answers and final tables of sampled filters equal the oracle's.

The expected multisets are built on the host from the same seeded streams
(the counting one from the rank counts, so no 10^9-element sort is needed).
"""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

from oracle import brute
from paper_2212_09005_amd import inputs
from paper_2212_09005_amd.workloads import C3, C4, C5

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
        assert a.shape == b.shape, f"{what}: {name} shape {a.shape} vs {b.shape}"
        bad = np.nonzero(a != b)[0]
        assert len(bad) == 0, f"{what}: {name} differs in {len(bad)} places, first {int(bad[0])}"


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=U64).view(np.int64)).to("cuda")


def test_counting_full_size_one_batch():
    from paper_2212_09005_amd import qf

    w = C3
    q, r, n, U = w.q, w.r, w.n, w.universe
    note(f"counting: q={q} r={r}, {n} Zipf({w.s}) instances over 2^{w.universe_log2} values, one batch")
    t0 = time.time()
    ranks = w.ranks()
    keys = inputs.rank_to_key(ranks)
    note(f"instances drawn ({time.time() - t0:.0f}s)")
    f = qf.CQF(q, r)
    d = dev64(keys)
    f.insert(d)
    assert f.sync() == 0
    del d
    torch.cuda.empty_cache()
    note(f"gpu insert done ({time.time() - t0:.0f}s)")
    # the multiset, from how often each value was drawn
    cnt = np.bincount(ranks, minlength=U + 1).astype(U64)
    nz = np.nonzero(cnt)[0]
    fps = brute.fingerprints(inputs.rank_to_key(nz), q, r)
    ms = brute.multiset(fps, cnt[nz])
    assert int(ms[1].sum()) == n
    rc, lay = f.export()
    assert rc == 0
    ref = brute.layout(*ms, q, r)
    note(f"distinct values {len(nz)}, distinct fingerprints {len(ms[0])}, used slots {int(ref.header[5])}")
    compare(lay, ref, "after the one-batch insert")
    del lay, ref
    note(f"table after insert bit-exact ({time.time() - t0:.0f}s)")
    ck = inputs.rank_to_key(w.count_ranks())
    dck = dev64(ck)
    cfp = brute.fingerprints(ck, q, r)
    got = f.count(dck).cpu().numpy().view(U64)
    want = brute.counts_of(*ms, cfp)
    assert np.array_equal(got, want), f"counts differ at {int(np.count_nonzero(got != want))} keys"
    # delete a random quarter of the instances
    mask = w.delete_mask()
    dcnt = np.bincount(ranks[mask], minlength=U + 1).astype(U64)
    drop = keys[mask]
    del ranks, keys, mask
    nfd = torch.zeros(1, dtype=torch.int64, device="cuda")
    dd = dev64(drop)
    f.delete(dd, nfd)
    assert f.sync() == 0
    assert int(nfd.item()) == 0
    note(f"deleted {len(drop)} instances ({time.time() - t0:.0f}s)")
    del dd, drop
    left = cnt[nz] - dcnt[nz]
    keep = left > 0
    ms2 = brute.multiset(fps[keep], left[keep])
    rc, lay = f.export()
    assert rc == 0
    compare(lay, brute.layout(*ms2, q, r), "after the delete")
    del lay
    got2 = f.count(dck).cpu().numpy().view(U64)
    want2 = brute.counts_of(*ms2, cfp)
    assert np.array_equal(got2, want2), f"counts after delete differ at {int(np.count_nonzero(got2 != want2))} keys"
    note(f"table and counts after delete bit-exact ({time.time() - t0:.0f}s)")
    f.close()


def test_many_filters_full_shape():
    from paper_2212_09005_amd import qf

    w = C4
    t0 = time.time()
    b = w.build()
    qs, off, keys, fid = b["qs"], b["off"], b["keys"], b["fid"]
    note(f"many filters: {w.nf} filters, {len(keys)} fill keys, {1 << w.query_log2} queries")
    fs = [qf.CQF(int(q), w.r) for q in qs]
    st = qf.CQFSet(fs)
    st.insert(torch.from_numpy(fid).to("cuda"), dev64(keys))
    assert st.sync() == 0
    dqf = torch.from_numpy(b["qfid"]).to("cuda")
    dqk = dev64(b["qkeys"])
    got_q = st.query(dqf, dqk).cpu().numpy()
    got_c = st.count(dqf, dqk).cpu().numpy().view(U64)
    note(f"gpu fill + lookups done ({time.time() - t0:.0f}s)")
    assert got_q[b["present"]].all(), "a present key was not found"
    assert np.array_equal(got_q, (got_c > 0).astype(np.uint8))
    # 24 filters of every size, whole tables and the answers routed to them
    g = np.random.Generator(np.random.PCG64(77))
    sample = []
    for qv in range(w.qlo, w.qhi + 1):
        idx = np.nonzero(qs == qv)[0]
        sample += sorted(g.choice(idx, size=min(24, len(idx)), replace=False).tolist())
    assert len(sample) >= 256
    checked = 0
    for i in sample:
        q = int(qs[i])
        ms = brute.multiset(brute.fingerprints(keys[off[i]:off[i + 1]], q, w.r))
        rc, lay = fs[i].export()
        assert rc == 0
        compare(lay, brute.layout(*ms, q, w.r), f"filter {i} (q={q})")
        sel = np.nonzero(b["qfid"] == i)[0]
        want = brute.counts_of(*ms, brute.fingerprints(b["qkeys"][sel], q, w.r))
        assert np.array_equal(got_c[sel], want), f"filter {i}: counts differ"
        checked += len(sel)
    note(f"{len(sample)} filters bit-exact, {checked} of their routed answers exact ({time.time() - t0:.0f}s)")
    st.close()
    for f in fs:
        f.close()


def test_serving_full_shape_mix_equals_alone_and_oracle():
    from paper_2212_09005_amd import qf

    w = C5
    t0 = time.time()
    qs, rs = w.filters()
    fills = w.fill_keys(qs)
    note(f"serving: {w.nf} filters, {sum(len(k) for k in fills)} fill keys ({time.time() - t0:.0f}s)")
    srv = qf.Server(64 << 30, max_round_keys=1 << 22)
    ids = [srv.open(int(q), int(r)) for q, r in zip(qs, rs)]
    tag = 0
    for i, k in enumerate(fills):
        for a in range(0, len(k), 1 << 22):
            srv.submit(qf.QFS_INSERT, ids[i], k[a:a + (1 << 22)], tag)
            tag += 1
    done = {}
    while len(done) < tag:
        for t, s_ in srv.poll(4096, 100000):
            done[t] = s_
    assert all(v == 0 for v in done.values())
    note(f"filled through the server ({time.time() - t0:.0f}s)")
    reqs = w.requests(1500, 1, qs, fills)
    sizes = np.array([len(k) for _, _, k in reqs])
    assert sizes.max() > 4096, "some rounds must take the radix-sort path"
    base = tag
    outs = {}
    for k, (op, f, keys) in enumerate(reqs):
        outs[base + k] = srv.submit(op, ids[f], keys, base + k)
    tag = base + len(reqs)
    g = np.random.Generator(np.random.PCG64(78))
    by_size = np.argsort(qs)
    sample = sorted({int(by_size[0]), int(by_size[-1])}
                    | {int(i) for i in np.nonzero(rs == 8)[0][:1]} | {int(i) for i in np.nonzero(rs == 16)[0][:1]}
                    | {int(i) for i in g.choice(w.nf, size=4, replace=False)})
    exports = {}
    for i in sample:
        exports[i] = srv.export(ids[i], int(qs[i]), int(rs[i]), tag)
        tag += 1
    done = {}
    t_end = time.time() + 300
    while len(done) < len(reqs) + len(sample):
        assert time.time() < t_end, f"only {len(done)} completions"
        for t, s_ in srv.poll(4096, 100000):
            done[t] = s_
    assert all(v == 0 for v in done.values()), "a request failed"
    stats = srv.stats()
    note(f"served {len(reqs)} requests in {stats['rounds']} rounds ({time.time() - t0:.0f}s)")
    served = [outs[base + k] for k in range(len(reqs))]

    # alone: the same stream, one request at a time, on identically filled filters
    fs = [qf.CQF(int(q), int(r)) for q, r in zip(qs, rs)]
    buf = torch.empty(1 << 22, dtype=torch.int64, device="cuda")
    for i, k in enumerate(fills):
        for a in range(0, len(k), 1 << 22):
            part = k[a:a + (1 << 22)]
            buf[:len(part)].copy_(torch.from_numpy(part.view(np.int64)))
            fs[i].insert(buf[:len(part)])
    nfb = torch.zeros(1, dtype=torch.int64, device="cuda")
    alone = []
    for op, f, keys in reqs:
        d = dev64(keys)
        if op == qf.QFS_INSERT:
            fs[f].insert(d)
            alone.append(None)
        elif op == qf.QFS_DELETE:
            fs[f].delete(d, nfb)
            alone.append(None)
        else:
            alone.append(fs[f].query(d).cpu().numpy())
    for f in fs:
        assert f.sync() == 0
    assert int(nfb.item()) == 0
    for k, (op, f, keys) in enumerate(reqs):
        if op == qf.QFS_QUERY:
            assert np.array_equal(served[k], alone[k]), f"request {k} (filter {f}): served and alone differ"
    note(f"every answer equals the one-request-at-a-time run ({time.time() - t0:.0f}s)")

    # the oracle: per sampled filter, the count of a fingerprint at a request
    # is its fill count plus the instances inserted minus those deleted by the
    # filter's earlier requests (no delete asks for more than is stored)
    for i in sample:
        q, r = int(qs[i]), int(rs[i])
        ms0 = brute.multiset(brute.fingerprints(fills[i], q, r))
        ev_fp, ev_t, ev_d = [], [], []
        for k, (op, f, keys) in enumerate(reqs):
            if f != i or op == qf.QFS_QUERY:
                continue
            ev_fp.append(brute.fingerprints(keys, q, r))
            ev_t.append(np.full(len(keys), k, np.int64))
            ev_d.append(np.full(len(keys), 1 if op == qf.QFS_INSERT else -1, np.int64))
        ev_fp = np.concatenate(ev_fp) if ev_fp else np.zeros(0, U64)
        ev_t = np.concatenate(ev_t) if ev_t else np.zeros(0, np.int64)
        ev_d = np.concatenate(ev_d) if ev_d else np.zeros(0, np.int64)
        order = np.lexsort((ev_t, ev_fp))
        efp, et, ed = ev_fp[order], ev_t[order], ev_d[order]
        cum = np.concatenate([[0], np.cumsum(ed)])
        nq = 0
        for k, (op, f, keys) in enumerate(reqs):
            if f != i or op != qf.QFS_QUERY:
                continue
            pf = brute.fingerprints(keys, q, r)
            lo = np.searchsorted(efp, pf, side="left")
            hi = lo + np.zeros(len(pf), np.int64)
            # events of the same fingerprint before request k
            span = np.searchsorted(efp, pf, side="right")
            for j in np.nonzero(span > lo)[0]:
                hi[j] = lo[j] + np.searchsorted(et[lo[j]:span[j]], k, side="left")
            cnt = brute.counts_of(*ms0, pf).astype(np.int64) + (cum[hi] - cum[lo])
            assert (cnt >= 0).all()
            assert np.array_equal(served[k], (cnt > 0).astype(np.uint8)), f"request {k} on filter {i} differs from the oracle"
            nq += 1
        dm = brute.multiset(ev_fp[ev_d < 0])
        im = brute.multiset(ev_fp[ev_d > 0])
        msf, short = brute.merge_multisets(brute.merge_multisets(ms0, im), dm, subtract=True)
        assert short == 0
        compare(exports[i].layout(), brute.layout(*msf, q, r), f"served filter {i} (q={q}, r={r})")
        note(f"filter {i} (q={q}, r={r}): {nq} query requests and the final table equal the oracle")
    srv.close()
    for f in fs:
        f.close()
