"""GPU tests of captured batch calls (qf_graph_*) and of launch parameters (qf_tune, qf_set_tune,
qf_autotune_set).

A captured graph is replayed several times with eager work and synchronisations in between
(new keys copied into the captured buffers); every replay must give exactly what the oracle
gives for the same batch applied to the filter's current contents.  Launch parameters change
how the work is cut, never the result: under every tuning the tables and answers must equal
the oracle's bit for bit.
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


def test_graph_single_filter_replays():
    qf = _qf()
    note("graph: insert + query + count of one filter, 4 replays")
    q, r, n, nq = 15, 8, 3000, 4000  # 18,000 keys in 32,768 quotients at the end
    f = qf.CQF(q, r)
    o = oqf.OracleQF(q, r)
    base = inputs.uniform_keys(300, 6000)
    f.insert(dev(base))
    assert o.insert(base) == 0
    s = torch.cuda.Stream()
    K = torch.zeros(n, dtype=torch.int64, device="cuda")
    Q = torch.zeros(nq, dtype=torch.int64, device="cuda")
    out8 = torch.zeros(nq, dtype=torch.uint8, device="cuda")
    out64 = torch.zeros(nq, dtype=torch.int64, device="cuda")
    f.reserve(n)
    torch.cuda.synchronize()
    g = qf.Graph(s)
    with g:
        f.insert(K, stream=s.cuda_stream)
        f.query(Q, out8, stream=s.cuda_stream)
        f.count(Q, out64, stream=s.cuda_stream)
    seen = [base]
    for rep in range(4):
        batch = inputs.uniform_keys(310 + rep, n)
        if rep == 2:
            batch[: n // 2] = base[: n // 2]  # counts above one
        probe = np.concatenate([np.concatenate(seen)[:2000], inputs.absent_keys(320 + rep, nq - 2000)])
        with torch.cuda.stream(s):
            K.copy_(dev(batch))
            Q.copy_(dev(probe))
        g.launch()
        s.synchronize()
        assert f.sync() == 0
        assert o.insert(batch) == 0
        seen.append(batch)
        want = o.count(probe)
        assert np.array_equal(host(out64), want), f"replay {rep}: counts"
        assert np.array_equal(host(out8), (want > 0).astype(np.uint8)), f"replay {rep}: queries"
        # eager work on the same filter between replays
        eager = f.count(Q)
        torch.cuda.synchronize()
        assert np.array_equal(host(eager), want)
    check_filter(f, o, "after replays")
    g.close()


def test_graph_set_replays():
    qf = _qf()
    qs = [10, 11, 12, 13, 14]
    note(f"graph: set insert + set count over q={qs}, 3 replays")
    fs = [qf.CQF(q, 8) for q in qs]
    os_ = [oqf.OracleQF(q, 8) for q in qs]
    st = qf.CQFSet(fs)
    rng = np.random.Generator(np.random.PCG64(9))
    n = 4000
    w = np.array([2.0 ** q for q in qs])
    K = torch.zeros(n, dtype=torch.int64, device="cuda")
    F = torch.zeros(n, dtype=torch.int32, device="cuda")
    C = torch.zeros(n, dtype=torch.int64, device="cuda")
    st.reserve(n)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = qf.Graph(s)
    with g:
        st.insert(F, K, stream=s.cuda_stream)
        st.count(F, K, C, stream=s.cuda_stream)
    for rep in range(3):
        fid = rng.choice(len(qs), size=n, p=w / w.sum()).astype(np.int32)
        keys = inputs.uniform_keys(400 + rep, n)
        with torch.cuda.stream(s):
            K.copy_(dev(keys))
            F.copy_(dev_fid(fid))
        g.launch()
        s.synchronize()
        assert st.sync() == 0
        want = np.zeros(n, dtype=U64)
        for i, o in enumerate(os_):
            sel = fid == i
            if sel.any():
                assert o.insert(keys[sel]) == 0
                want[sel] = o.count(keys[sel])
        assert np.array_equal(host(C), want), f"replay {rep}: counts"
    for i, (f, o) in enumerate(zip(fs, os_)):
        check_filter(f, o, f"filter {i} after set replays")
    g.close()


def test_graph_refuses_what_it_cannot_capture():
    qf = _qf()
    note("graph: an unreserved batch is refused under capture")
    f = qf.CQF(12, 8)
    big = torch.zeros(1 << 18, dtype=torch.int64, device="cuda")  # above any reservation
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with pytest.raises(qf.QFError) as e:
        with qf.Graph(s):
            f.insert(big, stream=s.cuda_stream)
    assert e.value.code == qf.QF_ERR_ARG
    # the filter is untouched and still usable
    k = inputs.uniform_keys(5, 100)
    f.insert(dev(k))
    assert f.sync() == 0
    assert int(host(f.count(dev(k))).sum()) == 100


def test_graph_replays_across_the_epoch_wrap():
    # each replay inserts then deletes the same keys (two merge launches), so
    # the table returns to the base after every replay; 33,000 replays take
    # the pipeline's 16-bit look-back epoch through its wrap, where the
    # device clears the look-back words itself
    qf = _qf()
    note("graph: 66,000 merge launches through the epoch wrap")
    q, r = 10, 8
    f = qf.CQF(q, r)
    o = oqf.OracleQF(q, r)
    base = inputs.uniform_keys(500, 700)
    f.insert(dev(base))
    assert o.insert(base) == 0
    ks = inputs.uniform_keys(501, 16)
    K = dev(ks)
    NF = torch.zeros(1, dtype=torch.int64, device="cuda")
    f.reserve(16)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = qf.Graph(s)
    with g:
        f.insert(K, stream=s.cuda_stream)
        f.delete(K, NF, stream=s.cuda_stream)
    probe = dev(np.concatenate([base[:200], ks]))
    want = o.count(np.concatenate([base[:200], ks]))
    for rep in range(33000):
        g.launch()
        if rep % 8250 == 8249:
            s.synchronize()
            assert f.sync() == 0, f"replay {rep}"
            got = f.count(probe)
            torch.cuda.synchronize()
            assert np.array_equal(host(got), want), f"replay {rep}: counts"
            note(f"replay {rep + 1} ok")
    s.synchronize()
    assert f.sync() == 0
    assert int(host(NF)[0]) == 0
    check_filter(f, o, "after the wrap")
    # and a plain batch afterwards still lands exactly
    extra = inputs.uniform_keys(502, 50)
    f.insert(dev(extra))
    assert o.insert(extra) == 0
    check_filter(f, o, "batch after the wrap")
    g.close()


@pytest.mark.parametrize("tuning", [
    dict(region_log2=6),
    dict(region_log2=9, sort_tile=2048),
    dict(region_log2=11, sort_chunk=16384, lookup_keys_per_lane=2),
    dict(sort_tile=2048, sort_chunk=65536, lookup_keys_per_lane=4),
])
def test_set_parity_under_every_tuning(tuning):
    qf = _qf()
    qs = [8, 10, 12, 13, 15]
    note(f"set parity under tuning {tuning}")
    fs = [qf.CQF(q, 8) for q in qs]
    os_ = [oqf.OracleQF(q, 8) for q in qs]
    st = qf.CQFSet(fs)
    st.tune(**tuning)
    got_t = st.tuning()
    for k, v in tuning.items():
        if k != "region_log2":
            assert got_t[k] == v
    rng = np.random.Generator(np.random.PCG64(77))
    w = np.array([2.0 ** q for q in qs])
    allk, allf = [], []
    for b, n in enumerate([20000, 7, 3000]):
        fid = rng.choice(len(qs), size=n, p=w / w.sum()).astype(np.int32)
        keys = inputs.uniform_keys(600 + b, n)
        st.insert(dev_fid(fid), dev(keys))
        for i, o in enumerate(os_):
            if (fid == i).any():
                assert o.insert(keys[fid == i]) == 0
        allk.append(keys)
        allf.append(fid)
    assert st.sync() == 0
    for i, (f, o) in enumerate(zip(fs, os_)):
        check_filter(f, o, f"filter {i} under {tuning}")
    keys = np.concatenate(allk + [inputs.absent_keys(610, 5000)])
    fid = np.concatenate(allf + [rng.integers(0, len(qs), 5000).astype(np.int32)])
    want = np.zeros(len(keys), dtype=U64)
    for i, o in enumerate(os_):
        want[fid == i] = o.count(keys[fid == i])
    assert np.array_equal(host(st.count(dev_fid(fid), dev(keys))), want)
    assert np.array_equal(host(st.query(dev_fid(fid), dev(keys))), (want > 0).astype(np.uint8))
    # deletes under the same tuning
    nfound = torch.zeros(len(qs), dtype=torch.int64, device="cuda")
    dk, df = keys[::3], fid[::3]
    st.delete(dev_fid(df), dev(dk), nfound)
    short = np.zeros(len(qs), dtype=U64)
    for i, o in enumerate(os_):
        if (df == i).any():
            rc, sh = o.delete(dk[df == i])
            assert rc == 0
            short[i] = sh
    assert np.array_equal(host(nfound), short)
    for i, (f, o) in enumerate(zip(fs, os_)):
        check_filter(f, o, f"filter {i} after delete under {tuning}")


def test_single_filter_tuning_and_bad_fields():
    qf = _qf()
    note("single-filter tuning; invalid fields rejected")
    f = qf.CQF(16, 16)
    o = oqf.OracleQF(16, 16)
    f.tune(region_log2=8, sort_tile=2048, lookup_keys_per_lane=4)
    assert f.tuning()["region_log2"] == 8
    keys = inputs.uniform_keys(700, 50000)
    f.insert(dev(keys))
    assert o.insert(keys) == 0
    check_filter(f, o, "r=16 with 256-slot regions")
    for bad in (dict(region_log2=5), dict(region_log2=14), dict(sort_tile=1000), dict(sort_chunk=5000),
                dict(sort_chunk=1 << 17), dict(lookup_keys_per_lane=3)):
        with pytest.raises(qf.QFError):
            f.tune(**bad)
    assert f.tuning()["region_log2"] == 8  # unchanged by the rejected calls


def test_autotune_picks_valid_parameters():
    qf = _qf()
    rng = np.random.Generator(np.random.PCG64(5))
    qs = [int(q) for q in rng.integers(10, 15, size=64)]
    note(f"autotune for 64 filters, {sum(1 << q for q in qs)} quotients")
    t, ms = qf.autotune_set(qs, 8, 0.85, 1 << 18)
    assert 6 <= t["region_log2"] <= 13
    assert t["sort_tile"] in (2048, 4096)
    assert t["sort_chunk"] in (4096, 16384)
    assert t["lookup_keys_per_lane"] in (1, 2, 4)
    assert ms[0] > 0 and ms[1] > 0
    t2, ms2 = qf.autotune_set(qs, 8, 0.85, 1 << 18)  # cached
    assert t2 == t and ms2 == ms
