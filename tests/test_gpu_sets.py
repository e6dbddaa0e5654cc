"""GPU parity of filter sets (one pipeline of launches for many filters).

Each filter of a set must end up exactly as the sequential oracle that receives
that filter's share of every batch, in batch order: exported tables bit for
bit, lookups element by element, not-found tallies per filter.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import oqf
from paper_2212_09005_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.uint64


def _qf():
    from paper_2212_09005_amd import qf

    return qf


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=U64).view(np.int64)).to("cuda")


def dev_fid(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda")


def host(t) -> np.ndarray:
    return t.cpu().numpy().view(U64) if t.dtype == torch.int64 else t.cpu().numpy()


def note(msg: str):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def check_filter(f, o, what):
    rc, lay = f.export()
    assert rc == 0, f"{what}: deferred error {rc}"
    ref = o.export()
    for name in ("occ_words", "runend_words", "slots", "offsets", "header"):
        a = np.asarray(getattr(lay, name)).astype(U64)
        b = np.asarray(getattr(ref, name)).astype(U64)
        bad = np.nonzero(a != b)[0]
        assert len(bad) == 0, f"{what}: {name} differs at {len(bad)} places, first {int(bad[0])}"


class SetCase:
    """Filters of the given sizes, their oracles, and a seeded tagged key stream."""

    def __init__(self, qs, r, seed):
        qf = _qf()
        self.qs, self.r = list(qs), r
        self.fs = [qf.CQF(q, r) for q in self.qs]
        self.os = [oqf.OracleQF(q, r) for q in self.qs]
        self.set = qf.CQFSet(self.fs)
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.seed = seed

    def tagged(self, n, seed, weights=None):
        """n keys, each tagged with a filter drawn proportionally to 2^q (or `weights`)."""
        w = np.array([2.0 ** q for q in self.qs]) if weights is None else np.asarray(weights, float)
        fid = self.rng.choice(len(self.qs), size=n, p=w / w.sum()).astype(np.int32)
        keys = inputs.uniform_keys(seed, n)
        return fid, keys

    def insert(self, fid, keys):
        self.set.insert(dev_fid(fid), dev(keys))
        for i, o in enumerate(self.os):
            part = keys[fid == i]
            if len(part):
                assert o.insert(part) == 0

    def delete(self, fid, keys):
        nf = torch.zeros(len(self.fs), dtype=torch.int64, device="cuda")
        self.set.delete(dev_fid(fid), dev(keys), nf)
        want = np.zeros(len(self.fs), dtype=U64)
        for i, o in enumerate(self.os):
            part = keys[fid == i]
            if len(part):
                rc, short = o.delete(part)
                assert rc == 0
                want[i] = short
        return host(nf), want

    def check_all(self, what):
        assert self.set.sync() == 0, what
        for i, (f, o) in enumerate(zip(self.fs, self.os)):
            check_filter(f, o, f"{what}, filter {i} (q={self.qs[i]})")

    def check_lookups(self, fid, keys, what):
        want = np.zeros(len(keys), dtype=U64)
        for i, o in enumerate(self.os):
            sel = fid == i
            if sel.any():
                want[sel] = o.count(keys[sel])
        got_c = host(self.set.count(dev_fid(fid), dev(keys)))
        got_q = host(self.set.query(dev_fid(fid), dev(keys)))
        assert np.array_equal(got_c, want), f"{what}: counts"
        assert np.array_equal(got_q, (want > 0).astype(np.uint8)), f"{what}: queries"


@pytest.mark.parametrize("r", [8, 16])
def test_set_of_mixed_sizes_insert_lookup_delete(r):
    qs = [6, 7, 9, 10, 12, 13, 14, 16]
    note(f"set of {len(qs)} filters q={qs} r={r}")
    c = SetCase(qs, r, seed=100 + r)
    cap = sum(int(0.8 * (1 << q)) for q in qs)
    batches = [1, 5, 300, 4096, cap // 3]
    all_fid, all_keys = [], []
    for b, n in enumerate(batches):
        fid, keys = c.tagged(n, seed=1000 * r + b)
        # a few duplicates inside the batch
        if n > 10:
            fid = np.concatenate([fid, fid[:7]])
            keys = np.concatenate([keys, keys[:7]])
        c.insert(fid, keys)
        all_fid.append(fid)
        all_keys.append(keys)
        c.check_all(f"after set insert batch {b} ({len(keys)} keys)")
    fid = np.concatenate(all_fid)
    keys = np.concatenate(all_keys)
    probe_fid = np.concatenate([fid[:5000], c.tagged(3000, seed=77)[0]])
    probe = np.concatenate([keys[:5000], inputs.absent_keys(78, 3000)])
    c.check_lookups(probe_fid, probe, "mixed probe")
    # deletes: some present, some absent, some twice
    dsel = np.arange(0, len(keys), 3)
    dfid = np.concatenate([fid[dsel], fid[:50], c.tagged(200, seed=79)[0]])
    dkeys = np.concatenate([keys[dsel], keys[:50], inputs.absent_keys(80, 200)])
    got_nf, want_nf = c.delete(dfid, dkeys)
    assert np.array_equal(got_nf, want_nf)
    c.check_all("after set delete")
    c.check_lookups(probe_fid, probe, "probe after delete")


def test_set_interleaved_with_single_filter_calls():
    qs = [10, 11, 12]
    note("set calls interleaved with per-filter calls")
    c = SetCase(qs, 8, seed=7)
    fid, keys = c.tagged(2000, seed=11)
    c.insert(fid, keys)
    # per-filter insert into filter 1, then a set batch again
    extra = inputs.uniform_keys(12, 500)
    c.fs[1].insert(dev(extra))
    assert c.os[1].insert(extra) == 0
    fid2, keys2 = c.tagged(1500, seed=13)
    c.insert(fid2, keys2)
    c.check_all("interleaved")
    c.check_lookups(np.concatenate([fid, fid2]), np.concatenate([keys, keys2]), "interleaved lookups")


def test_set_full_filter_fails_alone():
    # filter 0 (q=6, 64 quotients + 80 extra slots) receives far more keys
    # than it can hold; its share fails, the others are applied
    qf = _qf()
    qs = [6, 12]
    note("one filter of a set overflows")
    c = SetCase(qs, 8, seed=21)
    n0 = 400
    fid = np.concatenate([np.zeros(n0, np.int32), np.ones(1000, np.int32)])
    keys = inputs.uniform_keys(22, len(fid), distinct=True)
    c.set.insert(dev_fid(fid), dev(keys))
    assert c.set.sync() == qf.QF_ERR_FULL
    assert c.os[1].insert(keys[fid == 1]) == 0
    for i, (f, o) in enumerate(zip(c.fs, c.os)):
        check_filter(f, o, f"after overflow, filter {i}")


def test_set_filter_index_out_of_range():
    qf = _qf()
    qs = [8, 9]
    note("filter index out of range")
    c = SetCase(qs, 8, seed=31)
    fid = np.array([0, 1, 2, 1, 7, 0], dtype=np.int32)
    keys = inputs.uniform_keys(32, len(fid))
    c.set.insert(dev_fid(fid), dev(keys))
    assert c.set.sync() == qf.QF_ERR_ARG
    for i, o in enumerate(c.os):
        assert o.insert(keys[fid == i]) == 0
    for i, (f, o) in enumerate(zip(c.fs, c.os)):
        check_filter(f, o, f"valid keys kept, filter {i}")
    got = host(c.set.count(dev_fid(fid), dev(keys)))
    assert got[2] == 0 and got[4] == 0 and got[0] == 1 and got[1] == 1
    assert c.set.sync() == qf.QF_ERR_ARG


def test_set_many_small_filters():
    # the many-small-filters pattern: 300 filters of 2^10..2^14 quotients,
    # filled to load 0.85 by three set batches
    rng = np.random.Generator(np.random.PCG64(5))
    qs = [int(q) for q in rng.integers(10, 15, size=300)]
    note(f"300 small filters, total {sum(1 << q for q in qs)} quotients")
    c = SetCase(qs, 8, seed=41)
    # exact per-filter fill counts, spread over three batches
    want = [int(0.85 * (1 << q)) for q in qs]
    fid = np.concatenate([np.full(w, i, np.int32) for i, w in enumerate(want)])
    fid = inputs.shuffle(42, fid)
    keys = inputs.uniform_keys(43, len(fid))
    for part in np.array_split(np.arange(len(fid)), 3):
        c.insert(fid[part], keys[part])
    c.check_all("many small filters")
    probe_fid = np.concatenate([fid[:20000], rng.integers(0, len(qs), 20000).astype(np.int32)])
    probe = np.concatenate([keys[:20000], inputs.absent_keys(44, 20000)])
    c.check_lookups(probe_fid, probe, "many small filters")


def test_set_updates_restricted_to_listed_filters():
    # batches that list the filters they touch merge only those; the others
    # must stay exactly as they were, across many launches (look-back epochs)
    qs = [12, 13, 14, 15, 16]
    note("restricted set updates")
    c = SetCase(qs, 8, seed=61)
    fid, keys = c.tagged(3000, seed=62)
    c.insert(fid, keys)  # a full launch first
    for step in range(40):
        active = sorted(set(int(x) for x in c.rng.choice(len(qs), size=2, replace=False)))
        n = int(c.rng.integers(1, 150))
        f2 = c.rng.choice(active, size=n).astype(np.int32)
        k2 = inputs.uniform_keys(7000 + step, n)
        if step % 5 == 4:
            # delete some of the present keys of the listed filters
            pres = np.concatenate([keys[fid == a] for a in active])
            pf = np.concatenate([np.full(int((fid == a).sum()), a, np.int32) for a in active])
            sel = c.rng.integers(0, len(pres), size=min(n, len(pres)))
            nf = torch.zeros(len(qs), dtype=torch.int64, device="cuda")
            c.set.delete(dev_fid(pf[sel]), dev(pres[sel]), nf, active=active)
            want = np.zeros(len(qs), dtype=U64)
            for a in active:
                part = pres[sel][pf[sel] == a]
                if len(part):
                    rc, short = c.os[a].delete(part)
                    assert rc == 0
                    want[a] = short
            assert np.array_equal(host(nf), want)
        else:
            c.set.insert(dev_fid(f2), dev(k2), active=active)
            for a in active:
                part = k2[f2 == a]
                if len(part):
                    assert c.os[a].insert(part) == 0
            fid = np.concatenate([fid, f2])
            keys = np.concatenate([keys, k2])
        if step % 10 == 9:
            c.check_all(f"after restricted step {step}")
    c.check_all("after restricted updates")
    c.check_lookups(fid[:5000], keys[:5000], "restricted updates")


@pytest.mark.parametrize("qs", [[12, 12, 12, 6], [13, 11, 10, 9, 8, 7]])
def test_set_invalid_indexes_among_many_keys(qs):
    # many keys over several sort work-groups, some with filter indexes out of
    # range (their composite key is all ones): they must sort after every valid
    # key in every radix pass and leave the valid keys' tables exact
    qf = _qf()
    note(f"invalid indexes among many keys, q={qs}")
    c = SetCase(qs, 8, seed=91)
    fid, keys = c.tagged(int(0.7 * sum(1 << q for q in qs)), seed=92)
    bad = c.rng.random(len(fid)) < 0.05
    fid = fid.copy()
    fid[bad] = len(qs) + c.rng.integers(0, 5, size=int(bad.sum())).astype(np.int32)
    c.set.insert(dev_fid(fid), dev(keys))
    assert c.set.sync() == qf.QF_ERR_ARG
    for i, o in enumerate(c.os):
        part = keys[fid == i]
        if len(part):
            assert o.insert(part) == 0
    for i, (f, o) in enumerate(zip(c.fs, c.os)):
        check_filter(f, o, f"filter {i} with invalid indexes in the batch")


def test_set_finish_over_several_work_groups():
    # a filter with more regions than one finish work-group sums (2^25
    # quotients: 4096 regions, two work-groups) beside a one-region filter;
    # the statistics words of the header must match after every batch
    qs = [25, 12]
    note(f"statistics summed by several work-groups, q={qs}")
    c = SetCase(qs, 8, seed=171)
    fid, keys = c.tagged(600_000, seed=172)
    c.insert(fid, keys)
    c.check_all("first batch")
    fid2, keys2 = c.tagged(400_000, seed=173)
    c.insert(np.concatenate([fid2, fid[:1000]]), np.concatenate([keys2, keys[:1000]]))
    c.check_all("second batch with repeats")
    got_nf, want_nf = c.delete(np.concatenate([fid[:5000], fid2[:100]]),
                               np.concatenate([keys[:5000], inputs.absent_keys(174, 100)]))
    assert np.array_equal(got_nf, want_nf)
    c.check_all("after deletes")


def test_set_errors_info_and_reserve():
    # per-filter deferred errors name the filter that overflowed and are
    # cleared by the read; the set's info and a reserved scratch hold
    qf = _qf()
    qs = [6, 12, 10]
    note("set errors, info, reserve")
    c = SetCase(qs, 8, seed=301)
    c.set.reserve(50_000)
    info = c.set.info()
    assert info["nf"] == 3 and info["r"] == 8
    assert info["regions"] >= len(qs) and info["device_bytes"] > 0
    # filter 0 (64 quotients + 80 extra slots) receives 400 distinct keys
    fid = np.concatenate([np.zeros(400, np.int32), np.ones(2000, np.int32), np.full(500, 2, np.int32)])
    keys = inputs.uniform_keys(302, len(fid), distinct=True)
    c.set.insert(dev_fid(fid), dev(keys))
    n, codes = c.set.errors()
    assert n == 1 and int(codes[0]) == qf.QF_ERR_FULL and int(codes[1]) == 0 and int(codes[2]) == 0
    n, codes = c.set.errors()
    assert n == 0 and not codes.any()
    for i in (1, 2):
        assert c.os[i].insert(keys[fid == i]) == 0
    for i, (f, o) in enumerate(zip(c.fs, c.os)):
        check_filter(f, o, f"after a partial overflow, filter {i}")
    assert c.set.info()["batches"] == 1
