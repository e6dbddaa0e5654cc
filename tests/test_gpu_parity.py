"""GPU parity: the HIP library (through its C ABI) against the CPU oracles.

Integer work, so every comparison is exact: the exported table bit for bit,
every query and count element by element, the not-found tally of deletes.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import brute, oqf
from paper_2212_09005_amd import inputs
from tests.helpers import keys_for_fingerprints

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.uint64


def _qf():
    from paper_2212_09005_amd import qf

    return qf


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=U64).view(np.int64)).to("cuda")


def host(t) -> np.ndarray:
    return t.cpu().numpy().view(U64) if t.dtype == torch.int64 else t.cpu().numpy()


def note(msg: str):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def same_layout(gpu_lay, ref) -> tuple[bool, str]:
    msgs = []
    for name in ("occ_words", "runend_words", "slots", "offsets", "header"):
        a = np.asarray(getattr(gpu_lay, name)).astype(U64)
        b = np.asarray(getattr(ref, name)).astype(U64)
        if a.shape != b.shape:
            msgs.append(f"{name} shape {a.shape} vs {b.shape}")
            continue
        bad = np.nonzero(a != b)[0]
        if len(bad):
            i = int(bad[0])
            msgs.append(f"{name}: {len(bad)} diffs, first at {i}: gpu {int(a[i]):#x} ref {int(b[i]):#x}")
    return not msgs, "; ".join(msgs)


def export_ok(f, ref, what=""):
    rc, lay = f.export()
    assert rc == 0, f"deferred error {rc} {what}"
    ok, msg = same_layout(lay, ref)
    assert ok, f"{what}: {msg}"
    return lay


class Model:
    """The definition oracle's multiset, updated batch by batch."""

    def __init__(self, q, r):
        self.q, self.r = q, r
        self.ms = (np.zeros(0, U64), np.zeros(0, U64))

    def insert(self, keys):
        self.ms = brute.merge_multisets(self.ms, brute.multiset(brute.fingerprints(keys, self.q, self.r)))

    def delete(self, keys):
        self.ms, short = brute.merge_multisets(
            self.ms, brute.multiset(brute.fingerprints(keys, self.q, self.r)), subtract=True)
        return short

    def layout(self):
        return brute.layout(self.ms[0], self.ms[1], self.q, self.r)

    def counts(self, keys):
        return brute.counts_of(self.ms[0], self.ms[1], brute.fingerprints(keys, self.q, self.r))


def test_worked_example_lookup_from_imported_table():
    note("worked example q=6 r=8 via qf_import")
    qf = _qf()
    fps = np.array([(3 << 8) | 7, (3 << 8) | 9, (4 << 8) | 0, (5 << 8) | 200, (63 << 8) | 5], dtype=U64)
    cnt = np.array([1, 2, 3, 1, 300], dtype=U64)
    o = oqf.OracleQF(6, 8)
    assert o.insert_fp_counts(fps, cnt) == 0
    f = qf.CQF(6, 8)
    f.load(o.export())
    export_ok(f, o.export(), "import/export round trip")
    probe_fps = np.array([(4 << 8), (3 << 8) | 9, (63 << 8) | 5, (5 << 8) | 200, (5 << 8) | 199, (6 << 8), 0,
                          (63 << 8) | 4, (63 << 8) | 6], dtype=U64)
    keys = keys_for_fingerprints(probe_fps, 6, 8)
    want = o.count(keys)
    got = host(f.count(dev(keys)))
    assert np.array_equal(got, want)
    assert np.array_equal(host(f.query(dev(keys))), (want > 0).astype(np.uint8))


@pytest.mark.parametrize("r", [8, 16])
def test_c1_single_batch_insert_and_lookups(r):
    q = 16
    note(f"C1 q={q} r={r}: 58982 distinct keys, one batch")
    qf = _qf()
    keys = inputs.uniform_keys(1, int(0.9 * (1 << q)), distinct=True)
    absent = inputs.absent_keys(2, 1 << 16)
    f = qf.CQF(q, r)
    f.insert(dev(keys))
    assert f.sync() == 0
    o = oqf.OracleQF(q, r)
    assert o.insert(keys) == 0
    ref = o.export()
    export_ok(f, ref, "C1 table")
    probe = np.concatenate([keys, absent])
    want = o.count(probe)
    assert np.array_equal(host(f.count(dev(probe))), want)
    assert np.array_equal(host(f.query(dev(probe))), (want > 0).astype(np.uint8))


@pytest.mark.parametrize("q,r", [(14, 8), (13, 16), (16, 8), (10, 8), (6, 16)])
def test_ragged_batches_with_duplicates(q, r):
    note(f"ragged batches q={q} r={r}")
    qf = _qf()
    rng = np.random.Generator(np.random.PCG64(q * 31 + r))
    base = inputs.uniform_keys(q + r, int(0.6 * (1 << q)))
    f = qf.CQF(q, r)
    m = Model(q, r)
    sizes = [s for s in (1, 7, 255, 256, 1000, 4097) if s < (1 << q) // 4] + [len(base) // 3]
    for i, sz in enumerate(sizes):
        keys = base[rng.integers(0, len(base), sz)]
        f.insert(dev(keys))
        m.insert(keys)
        export_ok(f, m.layout(), f"after batch {i} ({sz} keys)")
    probe = np.concatenate([base[:3000], inputs.absent_keys(q, 3000)])
    assert np.array_equal(host(f.count(dev(probe))), m.counts(probe))


@pytest.mark.parametrize("q,r", [(14, 8), (12, 16)])
def test_delete_parity_and_not_found(q, r):
    note(f"deletes q={q} r={r}")
    qf = _qf()
    keys = inputs.uniform_keys(40 + q, int(0.8 * (1 << q)))
    keys = np.concatenate([keys, keys[:500], keys[:20]])
    f = qf.CQF(q, r)
    m = Model(q, r)
    f.insert(dev(keys))
    m.insert(keys)
    export_ok(f, m.layout(), "before deletes")
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    batches = [keys[:100], np.concatenate([keys[:600], inputs.absent_keys(9, 333)]), keys[1000:5000],
               keys[::3]]
    expect_nf = 0
    for i, b in enumerate(batches):
        f.delete(dev(b), nf)
        expect_nf += m.delete(b)
        export_ok(f, m.layout(), f"after delete batch {i}")
        assert int(nf.item()) == expect_nf
    # deleting everything left empties the table
    f.delete(dev(keys), nf)
    m.delete(keys)
    lay = export_ok(f, m.layout(), "after deleting all")
    assert int(lay.header[5]) == 0 and not np.any(lay.slots)


def test_large_counts_and_remainder_zero():
    q, r = 12, 8
    note("large counts, remainder 0, counters across slots")
    qf = _qf()
    fps = np.array([(100 << 8) | 0, (100 << 8) | 1, (100 << 8) | 255, (101 << 8) | 0, (4095 << 8) | 7, (0 << 8) | 0],
                   dtype=U64)
    mult = [300, 3, 70000, 2, 256, 1000]
    keys = np.concatenate([np.repeat(keys_for_fingerprints(fps[i:i + 1], q, r, seed=i), m)
                           for i, m in enumerate(mult)])
    keys = inputs.shuffle(5, keys)
    f = qf.CQF(q, r)
    m = Model(q, r)
    for part in np.array_split(keys, 4):
        f.insert(dev(part))
        m.insert(part)
        export_ok(f, m.layout(), "counting batch")
    probe = keys_for_fingerprints(fps, q, r, seed=99)
    assert np.array_equal(host(f.count(dev(probe))), np.array(mult, dtype=U64))
    # partial deletes shrink the counters
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    dk = keys[:40000]
    f.delete(dev(dk), nf)
    short = m.delete(dk)
    export_ok(f, m.layout(), "after partial delete")
    assert int(nf.item()) == short == 0


@pytest.mark.parametrize("r", [8, 16])
def test_long_run_crossing_regions(r):
    # every fingerprint in a handful of quotients: runs longer than a region,
    # spilling through later regions; exercises the global-memory paths
    q = 15
    note(f"long runs crossing regions q={q} r={r}")
    qf = _qf()
    rng = np.random.Generator(np.random.PCG64(r))
    quots = np.array([5, 4000, 4001, 20000], dtype=U64)
    rems = rng.integers(0, 1 << r, size=24000, dtype=np.uint64)
    qs = quots[rng.integers(0, len(quots), size=len(rems))]
    fps = (qs << U64(r)) | rems
    keys = keys_for_fingerprints(fps, q, r, seed=3)
    background = inputs.uniform_keys(77, 6000)
    f = qf.CQF(q, r)
    m = Model(q, r)
    for i, part in enumerate((background, keys[:12000], keys[12000:])):
        f.insert(dev(part))
        m.insert(part)
        export_ok(f, m.layout(), f"long-run batch {i}")
    probe = np.concatenate([keys[:5000], background[:1000], inputs.absent_keys(1, 2000)])
    assert np.array_equal(host(f.count(dev(probe))), m.counts(probe))
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    f.delete(dev(keys[:15000]), nf)
    m.delete(keys[:15000])
    export_ok(f, m.layout(), "long-run delete")


def test_full_batch_is_all_or_nothing():
    q, r = 6, 8
    note("QF_ERR_FULL all or nothing, q=6")
    qf = _qf()
    P = 64 + brute.extra_slots(q)
    keys = keys_for_fingerprints(np.array([(60 << 8) | (i % 256) for i in range(P - 55)], dtype=U64), q, r)
    f = qf.CQF(q, r)
    f.insert(dev(keys[: P - 70]))
    assert f.sync() == 0
    rc, before = f.export()
    assert rc == 0
    f.insert(dev(keys[P - 70:]))
    assert f.sync() == qf.QF_ERR_FULL
    assert f.sync() == 0  # the error is reported once
    rc, after = f.export()
    assert rc == 0
    assert same_layout(after, before)[0]
    # the filter keeps working after the rejected batch
    small = keys[P - 70: P - 65]
    f.insert(dev(small))
    o = oqf.OracleQF(q, r)
    assert o.insert(np.concatenate([keys[: P - 70], small])) == 0
    export_ok(f, o.export(), "after a rejected batch")


def test_empty_and_tiny_batches():
    q, r = 8, 16
    note("empty and one-key batches")
    qf = _qf()
    f = qf.CQF(q, r)
    empty = torch.zeros(0, dtype=torch.int64, device="cuda")
    f.insert(empty)
    f.delete(empty)
    assert f.query(empty).numel() == 0
    k = inputs.uniform_keys(3, 1)
    f.insert(dev(k))
    f.insert(dev(k))
    o = oqf.OracleQF(q, r)
    o.insert(np.concatenate([k, k]))
    export_ok(f, o.export(), "two single-key batches")
    assert int(host(f.count(dev(k)))[0]) == 2


def test_history_independence_on_gpu():
    q, r = 12, 8
    note("permutations and re-batching give one table")
    qf = _qf()
    keys = inputs.uniform_keys(8, 3500)
    keys = np.concatenate([keys, keys[:300]])
    ref = None
    for seed in range(3):
        perm = inputs.shuffle(seed, keys)
        f = qf.CQF(q, r)
        for part in np.array_split(perm, 1 + 5 * seed):
            f.insert(dev(part))
        rc, lay = f.export()
        assert rc == 0
        if ref is None:
            ref = lay
        else:
            assert same_layout(lay, ref)[0]
    o = oqf.OracleQF(q, r)
    o.insert(keys)
    assert same_layout(ref, o.export())[0]


@pytest.mark.parametrize("q,r,batches", [(18, 16, 1), (16, 8, 3)])
def test_zipf_counting_scaled(q, r, batches):
    """Counting config at reduced size: Zipf(1.1) instances over a universe of
    2^(q-2) values, 0.9 * 2^q instances, then counts over the universe and a
    Bernoulli(0.25) delete of the inserted instances."""
    note(f"zipf counting q={q} r={r} batches={batches}")
    qf = _qf()
    n = int(0.9 * (1 << q))
    keys = inputs.zipf_keys(3, n, 1.1, 1 << (q - 2))
    f = qf.CQF(q, r)
    m = Model(q, r)
    for part in np.array_split(keys, batches):
        f.insert(dev(part))
        m.insert(part)
    export_ok(f, m.layout(), "zipf insert")
    probe = inputs.rank_to_key(inputs.sample_without_replacement(4, 1 << (q - 2), 1 << 14) + 1)
    assert np.array_equal(host(f.count(dev(probe))), m.counts(probe))
    dmask = inputs.bernoulli_mask(5, n, 0.25)
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    f.delete(dev(keys[dmask]), nf)
    short = m.delete(keys[dmask])
    export_ok(f, m.layout(), "zipf delete")
    assert int(nf.item()) == short == 0


def test_launch_timer_kind_selection():
    # the timer brackets only the selected kinds; results are unaffected
    q, r = 14, 8
    note("launch timer kind selection")
    qf = _qf()
    f = qf.CQF(q, r)
    o = oqf.OracleQF(q, r)
    keys = inputs.uniform_keys(5, 8000)
    assert qf.qf_profile_enable(f.h, True, kinds=("merge", "lookup")) == 0
    f.insert(dev(keys[:3000]))
    f.query(dev(keys))
    prof = qf.qf_profile_read(f.h)
    assert prof["merge"][1] == 1 and prof["lookup"][1] == 1
    assert all(prof[k][1] == 0 for k in prof if k not in ("merge", "lookup"))
    assert prof["merge"][0] > 0.0
    assert qf.qf_profile_enable(f.h, True) == 0  # every kind
    # more keys than one work-group sorts: radix passes and the reduction
    f.insert(dev(keys[3000:]))
    prof = qf.qf_profile_read(f.h)
    assert prof["merge"][1] == 1 and prof["sort_scatter"][1] >= 1 and prof["reduce"][1] == 1
    assert prof["lookup"][1] == 0
    # a small batch: one sort-and-reduce launch, counted as a scatter
    f.insert(dev(keys[:100]))
    prof = qf.qf_profile_read(f.h)
    assert prof["sort_scatter"][1] == 1 and prof["sort_hist"][1] == 0 and prof["reduce"][1] == 0
    assert qf.qf_profile_enable(f.h, False) == 0
    f.insert(dev(keys[:10]))
    assert all(n == 0 for _, n in qf.qf_profile_read(f.h).values())
    o.insert(keys)
    o.insert(keys[:100])
    o.insert(keys[:10])
    export_ok(f, o.export(), "after timed and untimed batches")


@pytest.mark.parametrize("r", [8, 16])
def test_batches_around_the_one_group_sort_limit(r):
    # 4096 keys are sorted and reduced by one work-group, 4097 by the radix
    # passes; both sides of the limit, with heavy duplicates and deletes
    q = 16
    note(f"batches of 4095/4096/4097 keys, r={r}")
    qf = _qf()
    rng = np.random.Generator(np.random.PCG64(4096 + r))
    base = inputs.uniform_keys(90 + r, 20000)
    f = qf.CQF(q, r)
    m = Model(q, r)
    for i, sz in enumerate((4096, 4097, 4095, 4096)):
        keys = base[rng.integers(0, 3000 if i % 2 else len(base), sz)]
        f.insert(dev(keys))
        m.insert(keys)
        export_ok(f, m.layout(), f"after insert batch {i} ({sz} keys)")
    for i, sz in enumerate((4096, 4097)):
        keys = np.concatenate([base[rng.integers(0, 5000, sz - 50)], inputs.absent_keys(91 + i, 50)])
        nf = torch.zeros(1, dtype=torch.int64, device="cuda")
        f.delete(dev(keys), nf)
        short = m.delete(keys)
        assert int(host(nf)[0]) == int(short), f"delete batch {i}: not-found tally"
        export_ok(f, m.layout(), f"after delete batch {i} ({sz} keys)")
    probe = np.concatenate([base[:4000], inputs.absent_keys(93, 4000)])
    assert np.array_equal(host(f.count(dev(probe))), m.counts(probe))


def test_load_sweep_to_095_at_the_bench_ratio():
    # the bench's batch-to-table ratio (2^22 keys per 2^28 slots) at 2^20
    # slots: batches of 2^14 uniform keys up to load 0.95, the table exact
    # after every fifth batch and at the end, then one bench step (insert,
    # query, count, delete) at load 0.95 checked against the oracle
    q, r = 20, 8
    note("load sweep to 0.95, q=20, batches of 2^14")
    qf = _qf()
    f = qf.CQF(q, r)
    o = oqf.OracleQF(q, r)
    batch = 1 << 14
    fill = inputs.uniform_keys(2095, int(0.95 * (1 << q)))
    parts = [fill[s:s + batch] for s in range(0, len(fill), batch)]
    for i, part in enumerate(parts):
        f.insert(dev(part))
        assert o.insert(part) == 0
        if i % 5 == 4 or i == len(parts) - 1:
            export_ok(f, o.export(), f"after batch {i} (load {(i + 1) * batch / (1 << q):.3f})")
    ins = inputs.uniform_keys(2096, batch)
    f.insert(dev(ins))
    assert o.insert(ins) == 0
    export_ok(f, o.export(), "after the step's insert at load 0.95")
    qk = inputs.mixed_queries(2097, fill, batch // 2, batch - batch // 2)
    want = o.count(qk)
    assert np.array_equal(host(f.count(dev(qk))), want)
    assert np.array_equal(host(f.query(dev(qk))), (want > 0).astype(np.uint8))
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    f.delete(dev(ins), nf)
    rc, short = o.delete(ins)
    assert rc == 0 and int(host(nf)[0]) == short == 0
    export_ok(f, o.export(), "after the step's delete")
