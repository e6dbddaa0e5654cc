"""The two-choice filter on the GPU (include/tcf.h) against its oracle
(oracle/tcf.py).

Bulk form (Sec. 4.2): a bulk result is a function of the table and the
batch's multiset of keys, so after every batch the exported blocks and the
backing table must equal the oracle's bit for bit, not-found counts must
agree, and lookups must give the same answers element by element.

Point form (Sec. 4, Algorithm 1, Sec. 4.1): keys land concurrently, so which
candidate an item took is not unique.  What is unique is checked exactly:
every inserted key is found, the lookups of any key agree with the oracle's
lookup on the exported table, held + backed items equal the successful
inserts, and at a load where no block reaches 3/4 (every item takes the
shortcut into its primary block) each block's tag multiset equals the
oracle's.  The rest is checked for validity: the exported table must admit an
assignment of the inserted items to their candidate blocks and backing
entries (oracle.tcf.point_table_valid).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import tcf as otcf
from paper_2212_09005_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = np.uint64


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=U64).view(np.int64)).cuda()


def T():
    from paper_2212_09005_amd import tcf

    return tcf


def bulk_compare(g, o, what):
    slots, bk = g.export()
    bad = np.argwhere(slots != o.blocks)
    assert len(bad) == 0, f"{what}: {len(bad)} slots differ, first at block {bad[0][0]}"
    n = len(o.backing)
    assert np.array_equal(bk[:n], o.backing), f"{what}: backing table differs"
    assert (bk[n:] == 0).all()
    info = g.info()
    assert info["backing_used"] == n and info["held"] == int((o.blocks != otcf.EMPTY_B).sum()), what


def unambiguous(keys, nb):
    """Keys with no other key sharing (tag, a candidate block) or the
    backing identity: each stored tag then belongs to one key, so deletes
    are unambiguous."""
    b1, b2, tag, _ = otcf.tcf_hash(keys, nb)
    a = (b1 << U64(16)) | tag
    b = (b2 << U64(16)) | tag
    both = np.concatenate([a, np.where(b1 == b2, U64(2**63) + np.arange(len(b), dtype=U64), b)])
    u, c = np.unique(both, return_counts=True)
    dup = set(u[c > 1].tolist())
    ok = np.array([(int(x) not in dup) and (int(y) not in dup) for x, y in zip(a, b)])
    return keys[ok]


@pytest.mark.parametrize("nb", [64, 1024, 8192])
def test_bulk_batches_equal_the_oracle(nb):
    tcf = T()
    note(f"bulk TCF batches nb={nb}")
    slots = nb * otcf.BB
    g, o = tcf.TCF(nb, tcf.TCF_BULK), otcf.BulkTCF(nb)
    k1 = inputs.uniform_keys(100 + nb, int(0.35 * slots))
    k2 = np.concatenate([inputs.uniform_keys(200 + nb, int(0.3 * slots)), k1[: len(k1) // 10]])
    k3 = inputs.uniform_keys(300 + nb, int(0.2 * slots))
    for i, k in enumerate((k1, k2, k3)):
        g.insert(dev(k))
        o.insert(k)
        assert g.sync() == 0
        bulk_compare(g, o, f"after insert batch {i}")
    present = np.concatenate([k1[:4000], k3[:4000]])
    probe = np.concatenate([present, inputs.absent_keys(nb, 20000)])
    got = g.query(dev(probe)).cpu().numpy().astype(bool)
    assert np.array_equal(got, o.query(probe))
    assert got[: len(present)].all()
    dk = np.concatenate([k1[: len(k1) // 2], k2[:100], inputs.absent_keys(7 + nb, 3000)])
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    g.delete(dev(dk), not_found=nf)
    want_nf = o.delete(dk)
    assert g.sync() == 0
    bulk_compare(g, o, "after the delete batch")
    assert int(nf.item()) == want_nf
    k4 = inputs.uniform_keys(400 + nb, int(0.12 * slots))
    g.insert(dev(k4))
    o.insert(k4)
    assert g.sync() == 0
    bulk_compare(g, o, "after the insert after the delete")
    # a batch that takes the table past full: refused by both, nothing changes
    from paper_2212_09005_amd import qf

    k5 = inputs.uniform_keys(500 + nb, int(0.3 * slots))
    with pytest.raises(otcf.TableFull):
        o.insert(k5)
    with pytest.raises(qf.QFError) as e:
        g.insert(dev(k5))
    assert e.value.code == qf.QF_ERR_FULL
    bulk_compare(g, o, "after a refused batch")
    g.close()


def test_bulk_backing_overflow_is_all_or_nothing():
    tcf = T()
    from paper_2212_09005_amd import qf
    from tests.test_oracle_tcf import find_keys

    note("bulk TCF: backing overflow")
    nb = 2
    g, o = tcf.TCF(nb, tcf.TCF_BULK), otcf.BulkTCF(nb)
    k1 = find_keys(nb, 97, b1=0, b2=1)
    k2 = find_keys(nb, 40, b1=0, b2=0)
    k3 = find_keys(nb, 60, b1=0, b2=0, exclude=k2)
    for k in (k1, k2):
        g.insert(dev(k))
        o.insert(k)
    bulk_compare(g, o, "two batches")
    with pytest.raises(qf.QFError) as e:
        g.insert(dev(k3))
    assert e.value.code == qf.QF_ERR_FULL
    bulk_compare(g, o, "the batch that overflows the backing table changed nothing")
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    g.delete(dev(np.concatenate([k2, k1])), not_found=nf)
    assert o.delete(np.concatenate([k2, k1])) == 0 and int(nf.item()) == 0
    bulk_compare(g, o, "all deleted")
    g.close()


@pytest.mark.parametrize("nb", [256, 4096])
def test_point_inserts_are_valid_and_found(nb):
    tcf = T()
    note(f"point TCF inserts nb={nb}")
    slots = nb * otcf.PB
    keys = inputs.uniform_keys(500 + nb, int(0.85 * slots))
    keys = inputs.shuffle(3, np.concatenate([keys, keys[:200]]))
    g = tcf.TCF(nb, tcf.TCF_POINT)
    st = torch.full((len(keys),), 7, dtype=torch.int32, device="cuda")
    g.insert(dev(keys), status=st)
    assert g.sync() == 0 and (st.cpu().numpy() == 0).all()
    blocks, bk = g.export()
    why = otcf.point_table_valid(blocks, bk, keys)
    assert why is None, why
    info = g.info()
    assert info["held"] + info["backing_used"] == len(keys)
    probe = np.concatenate([keys, inputs.absent_keys(nb, 50000)])
    got = g.query(dev(probe)).cpu().numpy().astype(bool)
    assert got[: len(keys)].all()
    assert np.array_equal(got, otcf.point_query(blocks, bk, probe))
    g.close()


def test_point_shortcut_load_gives_the_unique_table():
    tcf = T()
    nb = 4096
    note(f"point TCF below 3/4 fill nb={nb}")
    keys = inputs.uniform_keys(600, int(0.15 * nb * otcf.PB))
    o = otcf.PointTCF(nb)
    for k in keys:
        assert o.insert(int(k))
    held = ((o.blocks != 0) & (o.blocks != otcf.TOMB)).sum(1)
    assert held.max() < otcf.SHORT_P  # every item took the shortcut
    g = tcf.TCF(nb, tcf.TCF_POINT)
    g.insert(dev(keys))
    assert g.sync() == 0
    blocks, bk = g.export()
    assert np.array_equal(np.sort(blocks, axis=1), np.sort(o.blocks, axis=1))
    assert (bk == 0).all()
    g.close()


def test_point_deletes_and_reinserts():
    tcf = T()
    nb = 2048
    note(f"point TCF deletes nb={nb}")
    keys = unambiguous(inputs.uniform_keys(700, int(0.9 * nb * otcf.PB)), nb)
    absent = unambiguous(np.concatenate([keys, inputs.absent_keys(701, 4000)]), nb)[-1000:]
    assert len(np.intersect1d(absent, keys)) == 0
    g = tcf.TCF(nb, tcf.TCF_POINT)
    g.insert(dev(keys))
    assert g.sync() == 0
    half = keys[: len(keys) // 2]
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    g.delete(dev(np.concatenate([half, absent])), not_found=nf)
    assert g.sync() == 0
    assert int(nf.item()) == len(absent)
    rest = keys[len(keys) // 2:]
    blocks, bk = g.export()
    why = otcf.point_table_valid(blocks, bk, rest)
    assert why is None, why
    assert g.query(dev(rest)).cpu().numpy().all()
    # tombstones are reused
    g.insert(dev(half))
    assert g.sync() == 0
    blocks, bk = g.export()
    assert otcf.point_table_valid(blocks, bk, keys) is None
    assert g.info()["held"] + g.info()["backing_used"] == len(keys)
    g.close()


def test_point_one_key_many_times_and_a_full_table():
    tcf = T()
    from paper_2212_09005_amd import qf

    note("point TCF: one key 40 times; a table past full")
    nb = 16
    g = tcf.TCF(nb, tcf.TCF_POINT)
    key = inputs.uniform_keys(800, 1)
    many = np.repeat(key, 40)
    g.insert(dev(many))
    assert g.sync() == 0
    blocks, bk = g.export()
    assert otcf.point_table_valid(blocks, bk, many) is None
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    g.delete(dev(many), not_found=nf)
    assert g.sync() == 0 and int(nf.item()) == 0
    blocks, bk = g.export()
    assert ((blocks == 0) | (blocks == otcf.TOMB)).all()
    g.close()
    nb = 4
    g = tcf.TCF(nb, tcf.TCF_POINT)
    keys = inputs.uniform_keys(801, 400)
    st = torch.full((len(keys),), 7, dtype=torch.int32, device="cuda")
    g.insert(dev(keys), status=st)
    assert g.sync() == qf.QF_ERR_FULL
    s = st.cpu().numpy()
    assert set(np.unique(s)) <= {0, qf.QF_ERR_FULL} and (s == qf.QF_ERR_FULL).any()
    blocks, bk = g.export()
    assert otcf.point_table_valid(blocks, bk, keys[s == 0]) is None
    assert ((blocks != 0) & (blocks != otcf.TOMB)).all()  # every slot taken
    g.close()


@pytest.mark.slow
def test_bulk_at_2p24_slots_load_09():
    tcf = T()
    nb = 1 << 17
    note(f"bulk TCF nb={nb} to load 0.9 in two batches")
    g, o = tcf.TCF(nb, tcf.TCF_BULK), otcf.BulkTCF(nb)
    slots = nb * otcf.BB
    for i, frac in enumerate((0.5, 0.4)):
        k = inputs.uniform_keys(900 + i, int(frac * slots))
        g.insert(dev(k))
        o.insert(k)
        assert g.sync() == 0
    bulk_compare(g, o, "2^24 slots at load 0.9")
    g.close()
