"""Pins of the CPU oracles (no GPU).

Two independent oracles are kept: oracle/oqf.c, a plain sequential counting
quotient filter that inserts and deletes by shifting clusters (Sec. 5.1,
Sec. 6.4), and oracle/brute.py, which builds the canonical table straight from
the fingerprint multiset.  They are pinned to things other than themselves:
a published hash test vector, hand-worked encodings and tables (tests/golden),
the inverse of the hash, brute force, invariants, closed forms from the paper
and a binomial check of the false-positive rate.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import brute, oqf
from paper_2212_09005_amd import inputs
from tests.helpers import fin64_inverse, golden_lines, keys_for_fingerprints

U64 = np.uint64


# ---------------------------------------------------------------- hash ----
def test_fin64_matches_published_splitmix64_vector():
    gamma = 0x9E3779B97F4A7C15
    for line in golden_lines("splitmix64_seed0.txt"):
        k, want = line.split()
        z = (int(k) * gamma) & ((1 << 64) - 1)
        assert oqf.fin64(z) == int(want, 16)
        assert int(brute.fin64(np.array([z], dtype=U64))[0]) == int(want, 16)


def test_fin64_is_a_bijection():
    x = inputs.uniform_keys(11, 200_000) ^ (inputs.uniform_keys(12, 200_000) << U64(1))
    h = brute.fin64(x)
    assert np.array_equal(fin64_inverse(h), x)
    # the C oracle computes the same function
    for v in x[:200]:
        assert oqf.fin64(int(v)) == int(brute.fin64(np.array([v]))[0])


def test_fingerprint_split_low_bits():
    f = oqf.OracleQF(10, 8)
    keys = inputs.uniform_keys(3, 1000)
    fps = brute.fingerprints(keys, 10, 8)
    assert all(f.fingerprint(int(k)) == int(p) for k, p in zip(keys, fps))
    assert int(fps.max()) < (1 << 18)
    # crafted keys land on the requested fingerprints
    want = np.arange(0, 1 << 18, 997, dtype=U64)
    assert np.array_equal(brute.fingerprints(keys_for_fingerprints(want, 10, 8), 10, 8), want)


# ------------------------------------------------------ counter encoding ----
def test_counter_encoding_golden():
    n = 0
    for line in golden_lines("counter_encoding_r8.txt"):
        lhs, rhs = line.split(":")
        x, c = (int(v) for v in lhs.split())
        want = [int(v) for v in rhs.split()]
        assert oqf.encode_entry(8, x, c) == want, (x, c)
        assert brute.encode_entry(x, c, 8) == want, (x, c)
        assert oqf.decode_entry(8, want) == (x, c, len(want))
        n += 1
    assert n >= 15


@pytest.mark.parametrize("r", [2, 3, 4, 8, 16])
def test_counter_roundtrip_and_lengths(r):
    rng = np.random.Generator(np.random.PCG64(r))
    R = 1 << r
    xs = list(range(R)) if R <= 256 else list(rng.integers(0, R, 64)) + [0, 1, R - 1]
    counts = list(range(1, 300)) + [int(v) for v in rng.integers(300, 1 << 62, 40)] + [(1 << 64) - 1, (1 << 64) - 2]
    for x in xs:
        x = int(x)
        for c in counts:
            enc = brute.encode_entry(x, c, r)
            assert len(enc) == int(brute.entry_lengths(np.array([x]), np.array([c], dtype=U64), r)[0])
            assert all(0 <= v < R for v in enc)
            # decodes alone, and when followed by a larger remainder's entry
            assert brute._decode_py(enc, 0, r) == (x, c, len(enc))
            if x + 1 < R:
                run = enc + [x + 1]
                assert brute._decode_py(run, 0, r) == (x, c, len(enc))
    # the C oracle agrees with the Python encoder on a sample
    for x in xs[:: max(1, len(xs) // 16)]:
        for c in counts[::7]:
            assert oqf.encode_entry(r, int(x), c) == brute.encode_entry(int(x), c, r)


def test_slot_maximum_counts_without_extra_slots():
    # Sec. 6.7: increments of an entry below the slot maximum need no shifting
    # beyond the counter itself: with r = 8, counts 3..257 all fit in 3 or 4
    # slots, and counts 3..(x+2) fit in exactly 3.
    for c in range(3, 258):
        assert len(brute.encode_entry(200, c, 8)) in (3, 4)
    assert all(len(brute.encode_entry(200, c, 8)) == 3 for c in range(3, 203))


# ------------------------------------------------------ worked example ----
def _worked_example():
    entries, exp = [], {"slot": {}, "lookup": []}
    for line in golden_lines("worked_example_q6_r8.txt"):
        tag, *vals = line.split()
        vals = [int(v) for v in vals]
        if tag == "entry":
            entries.append(vals)
        elif tag == "slot":
            exp["slot"][vals[0]] = vals[1]
        elif tag == "lookup":
            exp["lookup"].append(vals)
        else:
            exp[tag] = vals
    return entries, exp


def _check_worked(L, exp):
    P = int(L.header[4])
    occ = np.nonzero(brute.bits(L.occ_words, 64))[0].tolist()
    ends = np.nonzero(brute.bits(L.runend_words, P))[0].tolist()
    assert occ == exp["occupied"]
    assert ends == exp["runends"]
    assert L.offsets.tolist() == exp["offsets"]
    assert {i: int(v) for i, v in enumerate(L.slots) if v} == exp["slot"]
    assert int(L.header[5]) == exp["used"][0]
    assert int(L.header[6]) == exp["distinct"][0]
    assert int(L.header[7]) == exp["total"][0]


def test_worked_example_both_oracles():
    entries, exp = _worked_example()
    fps = np.array([(qq << 8) | rr for qq, rr, _ in entries], dtype=U64)
    cnt = np.array([c for *_, c in entries], dtype=U64)
    f = oqf.OracleQF(6, 8)
    assert f.insert_fp_counts(fps, cnt) == oqf.OQF_OK
    _check_worked(f.export(), exp)
    _check_worked(brute.layout(*brute.multiset(fps, cnt), 6, 8), exp)
    # lookups through real keys that hash to the listed fingerprints
    for qq, rr, want in exp["lookup"]:
        key = keys_for_fingerprints(np.array([(qq << 8) | rr], dtype=U64), 6, 8)
        assert int(f.count(key)[0]) == want
        assert int(f.query(key)[0]) == (want > 0)


# ------------------------------------------- oracle vs definition ---------
def _compare(f: oqf.OracleQF, ms, q, r):
    L = f.export()
    B = brute.layout(ms[0], ms[1], q, r)
    assert L.equal(B), L.diff(B)
    brute.check_invariants(L, r)
    return L


@pytest.mark.parametrize("q,r,n,dup", [(6, 8, 40, 1), (8, 8, 230, 3), (10, 4, 900, 2), (12, 8, 3600, 1),
                                       (10, 16, 950, 5), (7, 2, 110, 4), (12, 3, 3000, 9)])
def test_oracle_equals_definition_random(q, r, n, dup):
    base = inputs.uniform_keys(q * 100 + r, n // dup + 1)
    rng = np.random.Generator(np.random.PCG64(q + r))
    keys = base[rng.integers(0, len(base), n)]
    f = oqf.OracleQF(q, r)
    ms = (np.zeros(0, U64), np.zeros(0, U64))
    for chunk in np.array_split(keys, 3):
        assert f.insert(chunk) == oqf.OQF_OK
        ms = brute.merge_multisets(ms, brute.multiset(brute.fingerprints(chunk, q, r)))
        _compare(f, ms, q, r)
    # counts and queries equal the multiplicities
    probe = np.concatenate([keys[:200], inputs.absent_keys(q + 1, 300)])
    want = brute.counts_of(ms[0], ms[1], brute.fingerprints(probe, q, r))
    assert np.array_equal(f.count(probe), want)
    assert np.array_equal(f.query(probe), (want > 0).astype(np.uint8))


def test_adversarial_same_quotient_and_remainder_zero():
    q, r = 8, 8
    f = oqf.OracleQF(q, r)
    # every fingerprint in quotient 200: one long run that spills into the
    # extra slots; remainder 0 with large counts; remainder 255
    fps = np.array([(200 << 8) | x for x in range(0, 256, 5)] + [(250 << 8), (255 << 8) | 255], dtype=U64)
    cnt = np.array([1 + (i * 37) % 600 for i in range(len(fps))], dtype=U64)
    cnt[0] = 1 << 40
    assert f.insert_fp_counts(fps, cnt) == oqf.OQF_OK
    L = _compare(f, brute.multiset(fps, cnt), q, r)
    assert brute.clusters(L).max() > 64
    keys = keys_for_fingerprints(fps, q, r)
    assert np.array_equal(f.count(keys), cnt)


def test_full_is_all_or_nothing():
    q, r = 6, 8
    f = oqf.OracleQF(q, r)
    P = f.P
    keys = keys_for_fingerprints(np.array([(60 << 8) | (i % 256) for i in range(P - 55)], dtype=U64), q, r)
    assert f.insert(keys[: P - 70]) == oqf.OQF_OK
    before = f.export()
    assert f.insert(keys[P - 70 :]) == oqf.OQF_ERR_FULL  # last run would pass slot P-1
    assert f.export().equal(before)
    with pytest.raises(brute.TableFull):
        brute.layout(*brute.multiset(brute.fingerprints(keys, q, r)), q, r)


def test_count_overflow_is_all_or_nothing():
    f = oqf.OracleQF(8, 8)
    fps = np.array([77, 78], dtype=U64)
    assert f.insert_fp_counts(fps, np.array([(1 << 64) - 2, 5], dtype=U64)) == oqf.OQF_OK
    before = f.export()
    keys = keys_for_fingerprints(np.array([78, 77, 77], dtype=U64), 8, 8)
    assert f.insert(keys) == oqf.OQF_ERR_COUNT_OVERFLOW
    assert f.export().equal(before)


def test_history_independence():
    q, r = 10, 8
    keys = inputs.uniform_keys(5, 850)
    keys = np.concatenate([keys, keys[:100], keys[:10]])
    ref = oqf.OracleQF(q, r)
    assert ref.insert(keys) == 0
    L0 = ref.export()
    for seed in range(3):
        perm = inputs.shuffle(seed, keys)
        f = oqf.OracleQF(q, r)
        for part in np.array_split(perm, 1 + seed * 4):
            assert f.insert(part) == 0
        assert f.export().equal(L0)


def test_insert_delete_roundtrips():
    q, r = 10, 8
    A = inputs.uniform_keys(21, 500)
    B = inputs.uniform_keys(22, 300)
    f = oqf.OracleQF(q, r)
    assert f.insert(A) == 0
    empty = oqf.OracleQF(q, r).export()
    rc, nf = f.delete(A)
    assert (rc, nf) == (0, 0)
    assert f.export().equal(empty)
    g = oqf.OracleQF(q, r)
    assert g.insert(np.concatenate([A, B, B[:50]])) == 0
    rc, nf = g.delete(np.concatenate([B, B[:50]]))
    assert (rc, nf) == (0, 0)
    h = oqf.OracleQF(q, r)
    assert h.insert(A) == 0
    assert g.export().equal(h.export())


def test_delete_shortfall_and_saturation():
    q, r = 8, 8
    f = oqf.OracleQF(q, r)
    k = inputs.uniform_keys(31, 20)
    assert f.insert(np.concatenate([k, k[:5]])) == 0
    absent = inputs.absent_keys(32, 7)
    rc, nf = f.delete(np.concatenate([k[:5], k[:5], k[:5], absent]))
    # keys k[:5] held twice: the third deletion of each is a shortfall
    fps_abs = brute.fingerprints(absent, q, r)
    fps_k = brute.fingerprints(k, q, r)
    collide = int(np.isin(fps_abs, fps_k[5:]).sum())
    assert rc == 0 and nf == 5 + 7 - collide
    assert np.all(f.count(k[:5]) == brute.counts_of(*brute.multiset(fps_k[5:]), fps_k[:5]))


# ---------------------------------------------- C1-scale properties -------
def test_c1_config_no_false_negatives_and_fp_rate():
    """q=16, r=8: 58,982 distinct keys (load 0.9), 65,536 absent lookups."""
    q, r = 16, 8
    n = int(0.9 * (1 << q))
    keys = inputs.uniform_keys(1, n, distinct=True)
    absent = inputs.absent_keys(2, 1 << 16)
    f = oqf.OracleQF(q, r)
    assert f.insert(keys) == 0
    ms = brute.multiset(brute.fingerprints(keys, q, r))
    L = _compare(f, ms, q, r)
    assert np.all(f.query(keys) == 1)  # no false negatives (Sec. 1)
    cnt = f.count(keys)
    assert np.all(cnt >= 1)  # counts never under-estimate
    fp_abs = brute.fingerprints(absent, q, r)
    got = f.query(absent)
    assert np.array_equal(got, np.isin(fp_abs, ms[0]).astype(np.uint8))
    # statistical: P(false positive) = 1 - (1 - 2^-p)^D, D distinct fingerprints
    D = len(ms[0])
    p = 1.0 - (1.0 - 2.0 ** -(q + r)) ** D
    m = len(absent)
    mean, sd = m * p, math.sqrt(m * p * (1 - p))
    assert abs(int(got.sum()) - mean) < 3.3 * sd
    assert abs(p - 0.9 * 2 ** -8) < 3e-4  # ~ alpha * 2^-r
    # the paper's 8192-slot regions rely on clusters shorter than 8192 (Sec. 5.2)
    assert brute.clusters(L).max() < 8192


@pytest.mark.parametrize("q,r,load", [(10, 8, 0.95), (12, 16, 0.9), (14, 8, 0.99)])
def test_max_cluster_against_slot_scan(q, r, load):
    # the longest stretch of used slots, three ways: the C oracle's scan of its
    # own used bits, the vectorised cluster lengths of the canonical layout,
    # and a plain walk over the slots marked used by the runs [start, end]
    keys = inputs.uniform_keys(71 + q, int(load * (1 << q)))
    o = oqf.OracleQF(q, r)
    assert o.insert(keys) == 0
    L = o.export()
    P = int(L.header[4])
    used = np.zeros(P, dtype=bool)
    prev = -1
    ends = iter(np.nonzero(brute.bits(L.runend_words, P))[0])
    for x in np.nonzero(brute.bits(L.occ_words, 1 << q))[0]:
        e = int(next(ends))
        used[max(int(x), prev + 1): e + 1] = True
        prev = e
    best = cur = 0
    for u in used:
        cur = cur + 1 if u else 0
        best = max(best, cur)
    cl = brute.clusters(L)
    assert o.max_cluster() == best == int(cl.max())
    assert int(cl.sum()) == int(used.sum()) == int(L.header[5])


def test_import_of_the_definition_layout_continues_like_inserts():
    # a table loaded from brute.layout, then updated by the oracle, equals
    # the table the oracle builds by inserting everything itself
    q, r = 12, 8
    keys = inputs.uniform_keys(81, int(0.9 * (1 << q)))
    more = inputs.uniform_keys(82, 300)
    a = oqf.OracleQF(q, r)
    a.load(brute.layout(*brute.multiset(brute.fingerprints(keys, q, r)), q, r))
    assert a.max_cluster() == int(brute.clusters(a.export()).max())
    assert a.insert(more) == 0
    assert a.delete(keys[:500]) == (0, 0)
    b = oqf.OracleQF(q, r)
    assert b.insert(keys) == 0 and b.insert(more) == 0 and b.delete(keys[:500]) == (0, 0)
    assert a.export().equal(b.export())
    bad = brute.layout(*brute.multiset(brute.fingerprints(keys[:10], q, r)), q, r)
    bad.runend_words[-1] |= np.uint64(1) << np.uint64(63)
    with pytest.raises(ValueError):
        oqf.OracleQF(q, r).load(bad)


def test_cluster_bound_closed_form():
    # Sec. 5.2: longest cluster O(ln 2^q / (alpha - ln alpha - 1)); the paper's
    # example q = 40, alpha = 3/4 gives 736 slots.
    a = 0.75
    assert round(40 * math.log(2) / (a - math.log(a) - 1)) == 736


def test_bits_per_item_closed_form():
    # Table 3 lists 10.68 bits per item for the GQF with r = 8; the logical
    # table stores r remainder bits, one occupied and one run-end bit per slot
    # and an 8-bit offset per 64 slots: (8 + 2 + 8/64) / 10.68 = 0.948 load.
    per_slot = 8 + 2 + 8 / 64
    assert abs(per_slot / 0.948 - 10.68) < 0.005
    assert brute.extra_slots(16) == 2560 and brute.extra_slots(28) == 163840 and brute.extra_slots(30) == 327680
    assert oqf.extra_slots(16) == 2560 and oqf.extra_slots(6) == 128


def test_inputs_are_deterministic_and_disjoint():
    a = inputs.uniform_keys(1, 1000, distinct=True)
    assert np.array_equal(a, inputs.uniform_keys(1, 1000, distinct=True))
    assert len(np.unique(a)) == 1000
    b = inputs.absent_keys(2, 1000)
    assert not np.any(np.isin(a, b))
    z = inputs.zipf_ranks(3, 20000, 1.1, 1 << 28)
    assert z.min() >= 1 and z.max() <= (1 << 28)
    # head frequency of a Zipf(1.1) stream: P(1) = 1 / H, H = sum k^-1.1
    H = sum(k ** -1.1 for k in range(1, 200000)) + (200000 ** -0.1) / 0.1
    assert abs((z == 1).mean() - 1 / H) < 0.02


def test_zipf_sampler_matches_the_distribution():
    # rank frequencies of 2^24 draws against P(k) = k^-s / H(s, 2^28) in bins
    # (chi-square, 9 degrees of freedom, 99.9% critical value 27.9); H is summed
    # exactly to 10^6 and the rest by the Euler-Maclaurin integral
    s, U = 1.1, 1 << 28
    z = inputs.zipf_ranks(3, 1 << 24, s, U)
    assert z.min() >= 1 and z.max() <= U
    ks = np.arange(1, 10 ** 6 + 1, dtype=np.float64)
    w = ks ** -s
    a = 1 - s
    tail = ((U + 0.5) ** a - (10 ** 6 + 0.5) ** a) / a
    Hs = w.sum() + tail
    edges = [1, 2, 3, 4, 6, 11, 101, 10 ** 4 + 1, 10 ** 6 + 1, U + 1]
    cum = np.concatenate([[0.0], np.cumsum(w)])
    probs = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        if hi <= 10 ** 6 + 1:
            probs.append((cum[hi - 1] - cum[lo - 1]) / Hs)
        else:
            probs.append(tail / Hs)
    probs = np.array(probs)
    assert abs(probs.sum() - 1) < 1e-9
    counts = np.histogram(z, bins=edges)[0]
    exp = probs * len(z)
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 27.9, (chi2, counts, exp)
    # the stream does not depend on how it is cut into chunks or threads
    assert np.array_equal(inputs.zipf_ranks(3, 5_000_000, s, U), z[:5_000_000])


def test_block_counts_match_brute_force():
    """changed_blocks / query_blocks (units of the algorithmic-bytes model)
    against a per-block, per-key Python loop on small tables."""
    q, r = 10, 8
    keys = inputs.uniform_keys(61, 800)
    more = inputs.uniform_keys(62, 60)
    ms0 = brute.multiset(brute.fingerprints(keys, q, r))
    ms1 = brute.merge_multisets(ms0, brute.multiset(brute.fingerprints(more, q, r)))
    L0 = brute.layout(*ms0, q, r)
    L1 = brute.layout(*ms1, q, r)
    P = int(L0.header[4])
    nb = P // 64
    occ0, occ1 = brute.bits(L0.occ_words, 1 << q), brute.bits(L1.occ_words, 1 << q)
    re0, re1 = brute.bits(L0.runend_words, P), brute.bits(L1.runend_words, P)
    changed = 0
    for b in range(nb):
        sl = slice(64 * b, 64 * b + 64)
        diff = (np.any(L0.slots[sl] != L1.slots[sl]) or np.any(re0[sl] != re1[sl])
                or L0.offsets[b] != L1.offsets[b] or (64 * b < (1 << q) and np.any(occ0[sl] != occ1[sl])))
        changed += bool(diff)
    assert brute.changed_blocks(L0, L1) == changed
    # query blocks: home block, plus the blocks of the run found by walking runs
    probe = np.concatenate([keys[:100], inputs.absent_keys(63, 100)])
    fps = brute.fingerprints(probe, q, r)
    runs = {}
    prev = -1
    ends = iter(np.nonzero(re1)[0])
    for x in np.nonzero(occ1)[0]:
        e = int(next(ends))
        runs[int(x)] = (max(int(x), prev + 1), e)
        prev = e
    touched = set()
    for fp in fps:
        x = int(fp) >> r
        touched.add(x // 64)
        if x in runs:
            s, e = runs[x]
            touched.update(range(s // 64, e // 64 + 1))
    assert brute.query_blocks(L1, fps) == len(touched)


# ------------------------------------------------------- value association ----
def test_kv_lookup_by_hand_and_by_brute_force():
    # q = 2, r = 8, vbits = 3: a pair's fingerprint is the key's 7-bit
    # fingerprint (2 + 5 bits) then 3 value bits.  Keys crafted for key
    # fingerprints 0b0010110 and 0b1100001.
    q, r, v = 2, 8, 3
    ka = keys_for_fingerprints(np.array([0b0010110], dtype=U64), q, r - v, seed=1)[0]
    kb = keys_for_fingerprints(np.array([0b1100001], dtype=U64), q, r - v, seed=2)[0]
    keys = np.array([ka, ka, ka, kb, ka], dtype=U64)
    vals = np.array([5, 2, 5, 7, 11], dtype=U64)  # 11 mod 8 = 3
    fps = brute.kv_fingerprints(keys, vals, q, r, v)
    assert [int(x) for x in fps] == [0b0010110101, 0b0010110010, 0b0010110101, 0b1100001111, 0b0010110011]
    ufp, cnt = brute.multiset(fps)
    absent = keys_for_fingerprints(np.array([0b0010111], dtype=U64), q, r - v, seed=3)
    val, n = brute.kv_lookup(ufp, cnt, np.concatenate([[ka, kb], absent]), q, r, v)
    # key a holds values {2, 3, 5} (5 twice), key b holds {7}, the third none
    assert [int(x) for x in val] == [2, 7, 2**64 - 1] and list(n) == [3, 1, 0]
    # brute force over random pairs: per key fingerprint, the set of values
    g = np.random.Generator(np.random.PCG64(4))
    q, r, v = 6, 16, 5
    keys = inputs.uniform_keys(5, 300)[g.integers(0, 300, size=2000)]
    vals = g.integers(0, 1 << 12, size=2000).astype(U64)
    ufp, cnt = brute.multiset(brute.kv_fingerprints(keys, vals, q, r, v))
    fk = brute.fingerprints(keys, q, r - v)
    want = {}
    for k, x in zip(fk.tolist(), (vals & U64(31)).tolist()):
        want.setdefault(k, set()).add(x)
    probe = np.concatenate([keys[:500], inputs.absent_keys(6, 200)])
    val, n = brute.kv_lookup(ufp, cnt, probe, q, r, v)
    for k, x, c in zip(brute.fingerprints(probe, q, r - v).tolist(), val.tolist(), n.tolist()):
        s = want.get(k, set())
        assert c == len(s) and (x == min(s) if s else x == 2**64 - 1)


# ---- two layout facts the serving loop's in-place path relies on ----------

@pytest.mark.parametrize("q,load", [(8, 0.9), (10, 0.95), (10, 0.99), (12, 0.97)])
def test_used_slots_past_the_last_quotient_from_block_offset(q, load):
    # Slots at or past N are used only as one stretch from N that ends at the
    # table's last run end, and block N/64's offset gives it: off + 1 when
    # off > 0 or slot N ends a run, else 0.
    r = 8
    N = 1 << q
    seen = 0
    for seed in range(6):
        keys = inputs.uniform_keys(1000 * q + seed, int(load * N))
        ms = brute.multiset(brute.fingerprints(keys, q, r))
        lay = brute.layout(ms[0], ms[1], q, r)
        bits = np.unpackbits(np.asarray(lay.runend_words, dtype=np.uint64).view(np.uint8), bitorder="little")
        slots = np.asarray(lay.slots)
        ends = np.nonzero(bits)[0]
        t_true = max(0, int(ends.max()) + 1 - N) if len(ends) else 0
        # the stretch is contiguous: every slot of [N, N + t) holds something
        # of a run (a remainder or counter digit, possibly 0) and none after
        # it ends a run
        assert not bits[N + t_true:].any()
        off = int(np.asarray(lay.offsets)[N // 64])
        t = off + 1 if (off or bits[N]) else 0
        assert t == t_true, (seed, t, t_true)
        assert (slots[N + t_true:] == 0).all()
        seen += t_true > 0
    assert seen > 0 or load < 0.95


@pytest.mark.parametrize("rem", [0, 1, 77, 255])
def test_one_more_instance_adds_at_most_three_used_slots(rem):
    # the bound behind the in-place path's room test: each inserted key adds
    # at most 3 used slots (remainder 0 going from 2 to 3 copies adds 3)
    q, r = 8, 8
    prev, worst = 0, 0
    for c in range(1, 1500):
        lay = brute.layout(np.array([(5 << r) | rem], dtype=np.uint64), np.array([c], dtype=np.uint64), q, r)
        used = int(lay.header[5])
        worst = max(worst, used - prev)
        prev = used
    assert worst <= 3
    # and next to other runs the growth is the same: the run's own slots
    base = inputs.uniform_keys(9, 200)
    ms0 = brute.multiset(brute.fingerprints(base, q, r))
    u0 = int(brute.layout(ms0[0], ms0[1], q, r).header[5])
    extra = keys_for_fingerprints(np.array([(5 << r) | rem], dtype=np.uint64), q, r)
    ms1 = brute.merge_multisets(ms0, brute.multiset(brute.fingerprints(extra, q, r)))
    u1 = int(brute.layout(ms1[0], ms1[1], q, r).header[5])
    assert 0 <= u1 - u0 <= 3
