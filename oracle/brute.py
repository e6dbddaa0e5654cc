"""Counting quotient filter by definition, in numpy (the canonical layout).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this module.  It shares no code with the HIP
library, nor with oqf.c: the two oracles are independent implementations of
the same definition and are checked against each other.

What the filter holds is fixed by the paper without reference to any
algorithm:
  * Sec. 1 (footnote) and Sec. 5.1: the CQF is a lossless representation of
    the multiset h(S) of p-bit fingerprints; a query answers whether the
    fingerprint of x is in it, a count returns its multiplicity (which can only
    over-estimate the count of x itself).
  * Sec. 5.1: the fingerprint splits into quotient (canonical slot) and
    remainder; a run holds the remainders of one quotient, runs are stored in
    quotient order, each as far left as possible but not left of its quotient.
  * Sec. 5.3: remainders inside a run are sorted.
  * Sec. 5.4: equal fingerprints are one <item, count> entry.
Together with the readings taken where the paper is silent (SplitMix64 finalizer, low p
bits, CQF-style counter encoding, no wrap-around, 10*sqrt(2^q) extra slots,
offsets per 64-slot block), the table is a pure function of the multiset; this
module builds it directly: run ends satisfy
    end_i = max(quotient_i, end_{i-1} + 1) + length_i - 1,
which is evaluated in closed form with a running maximum.
"""
from __future__ import annotations

import numpy as np

from .oqf import Layout  # the plain container only; no arithmetic is shared

U64 = np.uint64
_MIX1 = U64(0xBF58476D1CE4E5B9)
_MIX2 = U64(0x94D049BB133111EB)


def fin64(keys: np.ndarray) -> np.ndarray:
    """SplitMix64 finalizer (Steele, Lea, Flood 2014), elementwise mod 2^64."""
    z = np.asarray(keys, dtype=U64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> U64(30)
        z *= _MIX1
        z ^= z >> U64(27)
        z *= _MIX2
        z ^= z >> U64(31)
    return z


def extra_slots(q: int) -> int:
    """Slots after slot 2^q - 1 where runs may still end: 64*ceil(10*isqrt(2^q)/64)."""
    import math

    e = 10 * math.isqrt(1 << q)
    return ((e + 63) // 64) * 64


def fingerprints(keys: np.ndarray, q: int, r: int) -> np.ndarray:
    """Low p = q + r bits of the hash (Sec. 5.1: p-bit fingerprint)."""
    h = fin64(keys)
    p = q + r
    if p >= 64:
        return h
    return h & U64((1 << p) - 1)


def multiset(fps: np.ndarray, counts: np.ndarray | None = None):
    """Sorted distinct fingerprints and their multiplicities (Sec. 5.4)."""
    fps = np.asarray(fps, dtype=U64)
    if counts is None:
        u, c = np.unique(fps, return_counts=True)
        return u.astype(U64), c.astype(U64)
    counts = np.asarray(counts, dtype=U64)
    order = np.argsort(fps, kind="stable")
    f = fps[order]
    c = counts[order]
    if len(f) == 0:
        return f, c
    head = np.ones(len(f), dtype=bool)
    head[1:] = f[1:] != f[:-1]
    idx = np.nonzero(head)[0]
    with np.errstate(over="ignore"):
        sums = np.add.reduceat(c, idx).astype(U64)
    return f[idx], sums


def merge_multisets(a, b, subtract: bool = False):
    """Multiset sum, or saturating difference a - b (returns also the shortfall)."""
    fa, ca = a
    fb, cb = b
    if not subtract:
        f = np.concatenate([fa, fb])
        c = np.concatenate([ca, cb])
        return multiset(f, c)
    pos = np.searchsorted(fa, fb)
    pos_c = np.minimum(pos, max(len(fa) - 1, 0))
    hit = (pos < len(fa)) & (fa[pos_c] == fb) if len(fa) else np.zeros(len(fb), dtype=bool)
    have = np.zeros(len(fb), dtype=U64)
    have[hit] = ca[pos_c[hit]]
    take = np.minimum(have, cb)
    shortfall = int((cb - take).sum())
    ca2 = ca.copy()
    ca2[pos_c[hit]] -= take[hit]
    keep = ca2 > 0
    return (fa[keep], ca2[keep]), shortfall


def _num_digits(v: np.ndarray, base: int) -> np.ndarray:
    nd = np.ones(len(v), dtype=np.int64)
    t = v // U64(base)
    while np.any(t > 0):
        nd += (t > 0)
        t = t // U64(base)
    return nd


def entry_lengths(rem: np.ndarray, cnt: np.ndarray, r: int) -> np.ndarray:
    """Slots taken by each (remainder, count) entry under the counter encoding."""
    rem = np.asarray(rem, dtype=U64)
    cnt = np.asarray(cnt, dtype=U64)
    base = (1 << r) - 1
    L = np.ones(len(rem), dtype=np.int64)
    L[cnt == 2] = 2
    big = cnt >= 3
    if np.any(big):
        v = cnt[big] - U64(3)
        nd = _num_digits(v, base)
        x = rem[big]
        msd = _msd_vec(v, nd, base)  # most significant base-(2^r-1) digit
        lead = (x > 0) & (msd >= x.astype(np.int64))
        L[big] = np.where(x > 0, 2 + nd + lead.astype(np.int64), 4 + nd)
    return L


def _msd_vec(v: np.ndarray, nd: np.ndarray, base: int) -> np.ndarray:
    out = np.zeros(len(v), dtype=np.int64)
    for k in np.unique(nd):
        m = nd == k
        out[m] = (v[m] // U64(base ** int(k - 1))).astype(np.int64)
    return out


def encode_entry(x: int, c: int, r: int) -> list[int]:
    """Slots of one entry (pure Python; used for entries with count >= 3)."""
    base = (1 << r) - 1
    if c == 1:
        return [x]
    if c == 2:
        return [x, x]
    v = c - 3
    digits = []
    while True:
        digits.append(v % base)
        v //= base
        if v == 0:
            break
    digits.reverse()
    if x > 0:
        body = [d if d < x else d + 1 for d in digits]
        if body[0] > x:
            body = [0] + body
        return [x] + body + [x]
    return [0, 0, 0] + [d + 1 for d in digits] + [0]


class TableFull(Exception):
    pass


def layout(ufp: np.ndarray, cnt: np.ndarray, q: int, r: int) -> Layout:
    """The canonical table of the multiset {ufp[i]: cnt[i]} (ufp sorted, distinct)."""
    N = 1 << q
    E = extra_slots(q)
    P = N + E
    ufp = np.asarray(ufp, dtype=U64)
    cnt = np.asarray(cnt, dtype=U64)
    quot = (ufp >> U64(r)).astype(np.int64)
    rem = ufp & U64((1 << r) - 1)
    lens = entry_lengths(rem, cnt, r)
    slots = np.zeros(P, dtype=np.uint16)
    runend = np.zeros(P, dtype=bool)
    occ = np.zeros(N, dtype=bool)
    offsets = np.zeros(P // 64, dtype=np.uint32)
    if len(ufp):
        head = np.ones(len(quot), dtype=bool)
        head[1:] = quot[1:] != quot[:-1]
        first = np.nonzero(head)[0]
        rq = quot[first]  # occupied quotients, ascending
        rl = np.add.reduceat(lens, first)  # run lengths
        S = np.cumsum(rl)
        S_prev = S - rl
        f = np.maximum.accumulate(np.maximum(rq - 1 - S_prev, -1))
        rend = f + S  # run ends
        rstart = rend - rl + 1
        if rend[-1] >= P:
            raise TableFull(f"last run ends at {int(rend[-1])} >= {P}")
        occ[rq] = True
        runend[rend] = True
        # entry start positions: run start + lengths of earlier entries in the run
        cl = np.cumsum(lens) - lens
        run_of = np.cumsum(head) - 1
        epos = rstart[run_of] + (cl - cl[first][run_of])
        one = cnt == 1
        slots[epos[one]] = rem[one]
        two = cnt == 2
        slots[epos[two]] = rem[two]
        slots[epos[two] + 1] = rem[two]
        for i in np.nonzero(cnt >= 3)[0]:
            enc = encode_entry(int(rem[i]), int(cnt[i]), r)
            slots[epos[i] : epos[i] + len(enc)] = enc
        # offsets (one per 64-slot block): run end of the last occupied
        # quotient <= block start, minus the block start, floored at 0
        bstart = np.arange(P // 64, dtype=np.int64) * 64
        k = np.searchsorted(rq, bstart, side="right")
        sel = np.where(k > 0, rend[np.maximum(k - 1, 0)], -1)
        offsets = np.maximum(sel - bstart, 0).astype(np.uint32)
    occ_words = np.packbits(occ, bitorder="little").view("<u8").astype(U64)
    rend_words = np.packbits(runend, bitorder="little").view("<u8").astype(U64)
    with np.errstate(over="ignore"):
        total = int(cnt.sum(dtype=U64)) if len(cnt) else 0
    header = np.array([q, r, N, E, P, int(lens.sum()), len(ufp), total], dtype=U64)
    return Layout(occ_words, rend_words, slots, offsets, header)


def kv_fingerprints(keys: np.ndarray, values: np.ndarray, q: int, r: int, vbits: int) -> np.ndarray:
    """Value association (the library's reading; the paper names the feature
    only): the key's fingerprint of q + r - vbits bits followed by the value's
    low vbits bits, a p = q + r bit fingerprint of the pair."""
    fk = fingerprints(keys, q, r - vbits)
    return (fk << U64(vbits)) | (np.asarray(values, dtype=U64) & U64((1 << vbits) - 1))


def kv_lookup(ufp: np.ndarray, cnt: np.ndarray, keys: np.ndarray, q: int, r: int, vbits: int):
    """Per key: the smallest value stored with its fingerprint (2^64 - 1 when
    none) and the number of distinct values, from the multiset {ufp: cnt} of
    pair fingerprints (the pairs of one key fingerprint fk are the fingerprints
    in [fk << vbits, (fk << vbits) + 2^vbits - 1])."""
    ufp = np.asarray(ufp, dtype=U64)
    lo = fingerprints(keys, q, r - vbits) << U64(vbits)
    hi = lo | U64((1 << vbits) - 1)
    a = np.searchsorted(ufp, lo, "left")
    b = np.searchsorted(ufp, hi, "right")
    n = (b - a).astype(np.int64)
    val = np.full(len(lo), np.iinfo(np.uint64).max, dtype=U64)
    hit = n > 0
    if len(ufp):
        val[hit] = ufp[a[hit]] & U64((1 << vbits) - 1)
    return val, n


def counts_of(ufp: np.ndarray, cnt: np.ndarray, fps: np.ndarray) -> np.ndarray:
    """Multiplicity of each queried fingerprint (0 when absent)."""
    fps = np.asarray(fps, dtype=U64)
    if len(ufp) == 0:
        return np.zeros(len(fps), dtype=U64)
    pos = np.searchsorted(ufp, fps)
    pos_c = np.minimum(pos, len(ufp) - 1)
    hit = (pos < len(ufp)) & (ufp[pos_c] == fps)
    out = np.zeros(len(fps), dtype=U64)
    out[hit] = cnt[pos_c[hit]]
    return out


def changed_blocks(a: Layout, b: Layout) -> int:
    """Number of 64-slot blocks whose slots, run ends, occupieds or offset differ."""
    nb = len(a.offsets)
    sa = a.slots.reshape(nb, 64)
    sb = b.slots.reshape(nb, 64)
    ch = np.any(sa != sb, axis=1)
    ch |= a.runend_words != b.runend_words
    ch |= a.offsets != b.offsets
    no = len(a.occ_words)
    ch[:no] |= a.occ_words != b.occ_words
    return int(ch.sum())


def run_bounds(L: Layout):
    """(occupied quotients, run starts, run ends) of a table, in quotient order."""
    q = int(L.header[0])
    occ = bits(L.occ_words, 1 << q)
    rq = np.nonzero(occ)[0].astype(np.int64)
    re = np.nonzero(bits(L.runend_words, int(L.header[4])))[0].astype(np.int64)
    prev = np.empty_like(re)
    if len(re):
        prev[0] = -1
        prev[1:] = re[:-1]
    rs = np.maximum(rq, prev + 1)
    return rq, rs, re


def query_blocks(L: Layout, fps: np.ndarray) -> int:
    """Distinct 64-slot blocks a batch of lookups must read: each key's home
    block (its occupied bit and offset) plus, when its quotient has a run, the
    blocks that hold that run."""
    r = int(L.header[1])
    nb = len(L.offsets)
    rq, rs, re = run_bounds(L)
    x = (np.asarray(fps, dtype=U64) >> U64(r)).astype(np.int64)
    mark = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(mark, x // 64, 1)
    np.add.at(mark, x // 64 + 1, -1)
    k = np.searchsorted(rq, x)
    kc = np.minimum(k, max(len(rq) - 1, 0))
    hit = (k < len(rq)) & (rq[kc] == x) if len(rq) else np.zeros(len(x), dtype=bool)
    np.add.at(mark, rs[kc[hit]] // 64, 1)
    np.add.at(mark, re[kc[hit]] // 64 + 1, -1)
    return int((np.cumsum(mark)[:nb] > 0).sum())


def bits(words: np.ndarray, n: int) -> np.ndarray:
    return np.unpackbits(np.asarray(words, dtype="<u8").view(np.uint8), bitorder="little")[:n].astype(bool)


def check_invariants(L: Layout, r: int) -> None:
    """Structural facts every canonical table satisfies (raises AssertionError)."""
    q = int(L.header[0])
    N = 1 << q
    P = int(L.header[4])
    occ = bits(L.occ_words, N)
    rend = bits(L.runend_words, P)
    rq = np.nonzero(occ)[0]
    re = np.nonzero(rend)[0]
    assert len(rq) == len(re), "one run end per occupied quotient"
    used = 0
    prev = -1
    total = 0
    distinct = 0
    inrun = np.zeros(P, dtype=bool)
    for x, e in zip(rq, re):
        s = max(int(x), prev + 1)
        assert e >= s >= x, "run lies at or after its quotient"
        inrun[s : e + 1] = True
        run = [int(v) for v in L.slots[s : e + 1]]
        p = 0
        last_rem = -1
        while p < len(run):
            xr, c, n = _decode_py(run, p, r)
            assert xr > last_rem, "remainders strictly ascending in a run"
            last_rem = xr
            total += c
            distinct += 1
            p += n
        used += e - s + 1
        prev = int(e)
    assert not np.any(L.slots[~inrun]), "slots outside runs are zero"
    assert used == int(L.header[5]) and distinct == int(L.header[6])
    assert (total % (1 << 64)) == int(L.header[7])
    bstart = np.arange(P // 64) * 64
    k = np.searchsorted(rq, bstart, side="right")
    sel = np.where(k > 0, re[np.maximum(k - 1, 0)] if len(re) else -1, -1)
    assert np.array_equal(np.maximum(sel - bstart, 0).astype(np.uint32), L.offsets), "offsets"


def _decode_py(run: list[int], p: int, r: int) -> tuple[int, int, int]:
    base = (1 << r) - 1
    x = run[p]
    e = len(run) - 1
    if x > 0:
        if p == e or run[p + 1] > x:
            return x, 1, 1
        if run[p + 1] == x:
            return x, 2, 2
        v, j = 0, p + 1
        while run[j] != x:
            d = run[j] if run[j] < x else run[j] - 1
            v = v * base + d
            j += 1
        return x, v + 3, j + 1 - p
    if p == e or run[p + 1] != 0:
        return 0, 1, 1
    if p + 1 == e or run[p + 2] != 0:
        return 0, 2, 2
    v, j = 0, p + 3
    while run[j] != 0:
        v = v * base + run[j] - 1
        j += 1
    return 0, v + 3, j + 1 - p


def clusters(L: Layout) -> np.ndarray:
    """Lengths of maximal runs of used slots (clusters, Sec. 5.1): a run that
    starts right after the previous run's end continues its cluster."""
    rq, rs, re = run_bounds(L)
    if len(rq) == 0:
        return np.zeros(0, dtype=np.int64)
    new_cluster = np.ones(len(rq), dtype=bool)
    new_cluster[1:] = rs[1:] > re[:-1] + 1
    first = np.nonzero(new_cluster)[0]
    last = np.r_[first[1:] - 1, len(rq) - 1]
    return (re[last] - rs[first] + 1).astype(np.int64)
