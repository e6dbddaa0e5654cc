"""Value association (qf_create_kv, qf_kv_insert_batch, qf_kv_delete_batch,
qf_kv_lookup_batch) against the definition oracle (oracle/brute.py).

The paper names value association among the CQF's features (Sec. 1, 2); the
library's reading stores each <key, value> pair as one fingerprint (the key's
fingerprint of q + r - vbits bits, then the value's bits), so the table must
equal, bit for bit, the canonical table of the pair multiset, and a lookup
must return exactly the smallest value and the number of distinct values the
oracle finds for the key's fingerprint.
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


def pairs(seed, nkeys, n, vbits):
    g = np.random.Generator(np.random.PCG64(seed))
    base = inputs.uniform_keys(seed, nkeys)
    keys = base[g.integers(0, nkeys, size=n)]
    vals = g.integers(0, 1 << (vbits + 2), size=n).astype(U64)  # values above 2^vbits wrap
    return keys, vals, base


def check_lookups(f, ms, probe, q, r, v, what):
    val, nv = f.kv_lookup(dev(probe))
    want_v, want_n = brute.kv_lookup(ms[0], ms[1], probe, q, r, v)
    assert np.array_equal(val.cpu().numpy().view(U64), want_v), what
    assert np.array_equal(nv.cpu().numpy().astype(np.int64), want_n), what


@pytest.mark.parametrize("q,r,v", [(14, 16, 8), (16, 8, 3), (12, 16, 1)])
def test_kv_batches_equal_the_oracle(q, r, v):
    from paper_2212_09005_amd import qf

    note(f"value association q={q} r={r} vbits={v}")
    f = qf.CQF.kv(q, r, v)
    k1, v1, base = pairs(1000 + q, int(0.3 * (1 << q)), int(0.5 * (1 << q)), v)
    f.kv_insert(dev(k1), dev(v1))
    assert f.sync() == 0
    ms = brute.multiset(brute.kv_fingerprints(k1, v1, q, r, v))
    rc, lay = f.export()
    compare(lay, brute.layout(*ms, q, r), "after the first batch")
    probe = np.concatenate([base[:3000], inputs.absent_keys(q, 3000)])
    check_lookups(f, ms, probe, q, r, v, "lookups after the first batch")
    # a second batch with pairs repeated and new ones (small-batch path too)
    k2, v2, _ = pairs(2000 + q, int(0.3 * (1 << q)), int(0.25 * (1 << q)), v)
    k2 = np.concatenate([k2, k1[:500]])
    v2 = np.concatenate([v2, v1[:500]])
    f.kv_insert(dev(k2), dev(v2))
    assert f.sync() == 0
    ms = brute.merge_multisets(ms, brute.multiset(brute.kv_fingerprints(k2, v2, q, r, v)))
    rc, lay = f.export()
    compare(lay, brute.layout(*ms, q, r), "after the second batch")
    check_lookups(f, ms, probe, q, r, v, "lookups after the second batch")
    # deletes of stored pairs, of pairs with a stored key but another value,
    # and of absent keys; the shortfall is counted
    dk = np.concatenate([k1[:2000], k1[:50], inputs.absent_keys(7, 100)])
    dv = np.concatenate([v1[:2000], v1[:50] + U64(1), np.zeros(100, dtype=U64)])
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    f.kv_delete(dev(dk), dev(dv), not_found=nf)
    assert f.sync() == 0
    ms, short = brute.merge_multisets(ms, brute.multiset(brute.kv_fingerprints(dk, dv, q, r, v)), subtract=True)
    rc, lay = f.export()
    compare(lay, brute.layout(*ms, q, r), "after the deletes")
    assert int(nf.item()) == short
    check_lookups(f, ms, probe, q, r, v, "lookups after the deletes")
    f.close()


def test_kv_resize_keeps_the_pairs_and_plain_calls_are_refused():
    from paper_2212_09005_amd import qf

    q, r, v = 14, 16, 4
    note(f"value association: resize ({q}, {r}) -> (22, 8), vbits {v}")
    f = qf.CQF.kv(q, r, v)
    k, vals, base = pairs(3000, 5000, 12000, v)
    f.kv_insert(dev(k), dev(vals))
    assert f.sync() == 0
    g = f.resize(22, 8)
    ms = brute.multiset(brute.kv_fingerprints(k, vals, q, r, v))
    rc, lay = g.export()
    compare(lay, brute.layout(*ms, 22, 8), "resized")
    probe = np.concatenate([base[:2000], inputs.absent_keys(9, 2000)])
    check_lookups(g, ms, probe, 22, 8, v, "lookups on the resized filter")
    for call in (lambda: f.insert(dev(k[:10])), lambda: f.delete(dev(k[:10])), lambda: f.query(dev(k[:10])),
                 lambda: f.count(dev(k[:10])), lambda: f.point_insert(dev(k[:10]))):
        with pytest.raises(qf.QFError) as e:
            call()
        assert e.value.code == qf.QF_ERR_ARG
    with pytest.raises(qf.QFError):
        qf.CQF.kv(q, 8, 8)  # no bits left for the key's remainder
    with pytest.raises(qf.QFError):
        f.resize(q + 12, r - 12)  # 4 remainder bits cannot hold 4 value bits and a key part
    f.close()
    g.close()
