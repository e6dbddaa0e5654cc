"""Enumeration, union, difference and re-layout of filters (qf_enumerate,
qf_merge_into, qf_resize) against the definition oracle (oracle/brute.py).

The paper names enumeration, merging and resizing as features of the counting
quotient filter (Sec. 1, 2) without describing them; the library's reading is
that they are exact operations on the stored fingerprint multiset, so every
result here must equal, bit for bit, the canonical table (or the sorted
<fingerprint, count> pairs) of the multiset the operation defines.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import brute
from paper_2212_09005_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.uint64


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=U64).view(np.int64)).cuda()


def compare(lay, ref, what):
    for name in ("occ_words", "runend_words", "slots", "offsets", "header"):
        a = np.asarray(getattr(lay, name)).astype(U64)
        b = np.asarray(getattr(ref, name)).astype(U64)
        bad = np.nonzero(a != b)[0]
        assert len(bad) == 0, f"{what}: {name} differs in {len(bad)} places, first {int(bad[0])}"


def skewed_keys(seed, n):
    """Keys with repeats of very different multiplicities (counts far above 2^r)."""
    g = np.random.Generator(np.random.PCG64(seed))
    base = inputs.uniform_keys(seed, max(8, n // 4))
    idx = np.minimum(g.zipf(1.3, size=n) - 1, len(base) - 1)
    return base[idx]


def built(q, r, keys):
    from paper_2212_09005_amd import qf

    f = qf.CQF(q, r)
    if len(keys):
        f.insert(dev(keys))
    assert f.sync() == 0
    return f


@pytest.mark.parametrize("q,r", [(14, 8), (13, 16), (18, 8)])
def test_enumerate_equals_the_multiset(q, r):
    note(f"enumerate q={q} r={r}")
    keys = np.concatenate([inputs.uniform_keys(600 + q, int(0.6 * (1 << q))), skewed_keys(700 + q, 1 << (q - 2))])
    f = built(q, r, keys)
    fp, cnt = f.enumerate()
    ms = brute.multiset(brute.fingerprints(keys, q, r))
    assert np.array_equal(fp.cpu().numpy().view(U64), ms[0])
    assert np.array_equal(cnt.cpu().numpy().view(U64), ms[1])
    st = f.stats()
    assert st["distinct"] == len(ms[0]) and st["total"] == int(ms[1].sum())
    f.close()


def test_enumerate_empty_and_too_small():
    from paper_2212_09005_amd import qf
    import ctypes

    f = qf.CQF(12, 8)
    fp, cnt = f.enumerate()
    assert fp.numel() == 0 and cnt.numel() == 0
    f.insert(dev(inputs.uniform_keys(5, 100)))
    n = ctypes.c_uint64(0)
    buf = torch.empty(10, dtype=torch.int64, device="cuda")
    rc = qf.lib().qf_enumerate(f.h, buf.data_ptr(), buf.data_ptr(), 10, ctypes.byref(n), None)
    assert rc == qf.QF_ERR_ARG and n.value == 100
    f.close()


@pytest.mark.parametrize("q,r", [(15, 8), (14, 16)])
def test_union_difference_and_self(q, r):
    note(f"union / difference q={q} r={r}")
    k1 = np.concatenate([inputs.uniform_keys(800, int(0.4 * (1 << q))), skewed_keys(801, 1 << (q - 3))])
    k2 = np.concatenate([inputs.uniform_keys(802, int(0.3 * (1 << q))), k1[: 1 << (q - 4)], skewed_keys(801, 99)])
    a, b = built(q, r, k1), built(q, r, k2)
    m1 = brute.multiset(brute.fingerprints(k1, q, r))
    m2 = brute.multiset(brute.fingerprints(k2, q, r))
    a.merge_from(b)
    assert a.sync() == 0
    rc, lay = a.export()
    u = brute.merge_multisets(m1, m2)
    compare(lay, brute.layout(*u, q, r), "union")
    rc, lb = b.export()
    compare(lb, brute.layout(*m2, q, r), "the source after the union")
    # difference: (m1 + m2) - m2 = m1; then minus m2 again: saturating, shortfall counted
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    a.merge_from(b, subtract=True, not_found=nf)
    assert a.sync() == 0 and int(nf.item()) == 0
    rc, lay = a.export()
    compare(lay, brute.layout(*m1, q, r), "difference back to the first multiset")
    a.merge_from(b, subtract=True, not_found=nf)
    assert a.sync() == 0
    d, short = brute.merge_multisets(m1, m2, subtract=True)
    rc, lay = a.export()
    compare(lay, brute.layout(*d, q, r), "saturating difference")
    assert int(nf.item()) == short
    # a filter merged with itself doubles every count
    b.merge_from(b)
    assert b.sync() == 0
    rc, lb = b.export()
    compare(lb, brute.layout(m2[0], m2[1] * U64(2), q, r), "self union")
    a.close()
    b.close()


def test_resize_both_ways_and_cross_split_union():
    note("resize (14, 16) -> (22, 8) -> (14, 16); union across splits")
    keys = np.concatenate([inputs.uniform_keys(900, 9000), skewed_keys(901, 4000)])
    src = built(14, 16, keys)
    ms = brute.multiset(brute.fingerprints(keys, 14, 16))
    big = src.resize(22, 8)
    rc, lay = big.export()
    assert rc == 0
    # the same p = 30 bit fingerprints, split 22 + 8
    compare(lay, brute.layout(ms[0], ms[1], 22, 8), "resized to q=22, r=8")
    back = big.resize(14, 16)
    rc, lay = back.export()
    compare(lay, brute.layout(ms[0], ms[1], 14, 16), "resized back")
    # union of filters with different splits of the same fingerprint length
    k2 = inputs.uniform_keys(902, 20000)
    other = built(22, 8, k2)
    other.merge_from(src)
    assert other.sync() == 0
    rc, lay = other.export()
    u = brute.merge_multisets(brute.multiset(brute.fingerprints(k2, 22, 8)), ms)
    compare(lay, brute.layout(*u, 22, 8), "union across splits")
    for f in (src, big, back, other):
        f.close()


@pytest.mark.slow
def test_resize_at_scale():
    note("resize (20, 16) at load 0.8 -> (28, 8)")
    q, r = 20, 16
    keys = inputs.uniform_keys(950, int(0.8 * (1 << q)))
    src = built(q, r, keys)
    ms = brute.multiset(brute.fingerprints(keys, q, r))
    big = src.resize(28, 8)
    rc, lay = big.export()
    assert rc == 0
    compare(lay, brute.layout(ms[0], ms[1], 28, 8), "resized to q=28")
    src.close()
    big.close()


def test_union_that_does_not_fit_leaves_the_destination_unchanged():
    from paper_2212_09005_amd import qf

    q, r = 10, 8
    a = built(q, r, inputs.uniform_keys(960, 900))
    b = built(q, r, inputs.uniform_keys(961, 700))
    rc, before = a.export()
    a.merge_from(b)
    assert a.sync() == qf.QF_ERR_FULL
    rc, after = a.export()
    compare(after, before, "a union past the last slot is not applied")
    with pytest.raises(qf.QFError):
        a.resize(12, 8)  # q + r must stay the same
    a.close()
    b.close()
