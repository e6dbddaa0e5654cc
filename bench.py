#!/usr/bin/env python3
"""Throughput of the counting quotient filter on one MI355X.

Workload (2^28 quotients, r = 8, load 0.9, batches of 2^22 uniform keys; see
paper_2212_09005_amd/workloads.py): the filter is filled to load 0.9 (not
timed); one step then runs the whole hot path on one batch -- insert 2^22
fresh keys, query 2^22 keys (half present, half absent), count the same keys,
delete the inserted batch -- which returns the table to load 0.9.  Inputs are
resident in HBM before the timed region.

Prints one JSON line: aggregate ops/s over the step (value), the per-operation
rates (insert and query from events between the operations of the timed
steps), the roofline of the dominant kernel measured with HIP events on its
launch stream, beside the attainable bandwidth of a device-to-device copy, and
the CPU oracle timed on a bounded sample of the same step at the same size.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
METRIC = "B inserts/s and B queries/s at load 0.9 (2^28 slots, r=8); % HBM roofline"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def to_dev(a: np.ndarray, torch):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to("cuda")


def load_constants(w) -> dict | None:
    path = os.path.join(ROOT, "tests", "golden", "bench_c2_constants.json")
    if not os.path.exists(path):
        return None
    c = json.load(open(path))
    if (c["q"], c["r"], c["load"], c["batch"]) != (w.q, w.r, w.load, w.batch):
        return None
    return c


def algorithmic_bytes(kind: str, w, consts: dict | None, lookup_count_share: float) -> float | None:
    """Bytes the method itself must move per launch of `kind`: a merge reads and writes each
    changed block once (at its information-theoretic size) and reads its distinct entries; a
    lookup reads its keys, writes its results and reads each distinct block it touches."""
    m = w.batch
    Bb = 64 * (w.r + 2) // 8 + 1
    if kind == "hash":
        return 8.0 * m  # read the keys
    if kind == "sort_scatter":
        return None  # charged to the grouping round trip below, not per pass
    if consts is None:
        return None
    if kind == "merge":
        # table read-modify-write of the changed blocks + the reduced batch read once
        return 2.0 * Bb * consts["C_mean"] + 16.0 * consts["u_mean"]
    if kind == "lookup":
        # keys in, one result out (1 B query, 8 B count), the distinct blocks read
        out_b = 1.0 * (1 - lookup_count_share) + 8.0 * lookup_count_share
        return (8.0 + out_b) * m + Bb * consts["D_mean"]
    return None


def measured_traffic(kernel: str) -> float | None:
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None when
    the kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_q28_r8_load0.9_batch2p22.md")
    if not os.path.exists(path):
        return None
    line = next((l for l in open(path) if l.startswith("traffic-json:")), None)
    if line is None:
        return None
    rec = json.loads(line.split(":", 1)[1]).get(kernel)
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_2212_09005_amd", "csrc", rec["src"])
    if hashlib.sha1(open(src, "rb").read()).hexdigest() != rec["sha1"]:
        return None
    return float(rec["bytes"])


def host_cpu() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(w, fill: np.ndarray, budget_s: float = 20.0, m: int = 1 << 18) -> dict:
    """The CPU oracle (oracle/oqf.c, one thread, as it stands) on the headline step at the headline
    size: the table of the same fill keys (built by the definition oracle and loaded, not timed),
    then steps of insert / query / count / delete with batches of m keys of the same streams
    (the first m keys of each step's batch), for about budget_s seconds."""
    from oracle import brute, oqf

    t0 = time.perf_counter()
    ms = brute.multiset(brute.fingerprints(fill, w.q, w.r))
    o = oqf.OracleQF(w.q, w.r)
    o.load(brute.layout(ms[0], ms[1], w.q, w.r))
    del ms
    t_load = time.perf_counter() - t0
    op_s = np.zeros(4)
    steps = 0
    while True:
        ins = w.insert_keys(steps)[:m]
        qk = w.query_keys(steps, fill)[:m]
        t = [time.perf_counter()]
        assert o.insert(ins) == 0
        t.append(time.perf_counter())
        o.query(qk)
        t.append(time.perf_counter())
        o.count(qk)
        t.append(time.perf_counter())
        rc, nf = o.delete(ins)
        t.append(time.perf_counter())
        assert rc == 0 and nf == 0
        op_s += np.diff(t)
        steps += 1
        if op_s.sum() > budget_s or steps >= 64:
            break
    total = float(op_s.sum())
    rates = {k: round(float(m * steps / op_s[i] / 1e9), 6)
             for i, k in enumerate(("insert", "query", "count", "delete"))}
    return {
        "value": round(4 * m * steps / total / 1e9, 6),
        "unit": "B ops/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle/oqf.c (sequential CQF, 1 thread) on the headline table (q={w.q}, r={w.r}, load {w.load}, "
                   f"loaded from the definition layout in {t_load:.0f}s, not timed): {steps} steps of insert / "
                   f"query / count / delete of {m} keys each (every insert also snapshots the table for "
                   f"all-or-nothing)"),
        "rates_Bps": rates,
        "host": host_cpu(),
    }


def host_threads() -> int:
    """Threads for the all-core oracle runs: the host's cores, at most 16 (one GPU's share of a
    shared host)."""
    return max(1, min(os.cpu_count() or 1, 16))


def shard(items, weight, threads: int) -> list:
    """Items spread over threads, heaviest first to the least-loaded thread."""
    shards, load = [[] for _ in range(threads)], [0] * threads
    for i in sorted(items, key=weight, reverse=True):
        t = load.index(min(load))
        shards[t].append(i)
        load[t] += weight(i)
    return shards


def pool_time(fn, shards, threads: int) -> float:
    """Wall seconds of fn over the shards on a pool of threads (the oracle's calls release the
    interpreter lock, so independent filters run in parallel)."""
    from concurrent.futures import ThreadPoolExecutor

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(fn, shards))
    return time.perf_counter() - t0


def cpu_baseline_sets(b: dict, nf: int, order, qoff, got_set, budget_keys: int = 1 << 25) -> dict:
    """The CPU oracle (oracle/oqf.c as it stands) on a sample of the many-filter workload, with
    independent filters spread over all host threads (one shard of filters per thread): every
    stride-th filter, about budget_keys fill keys in all, filled in one batch each and then asked
    its share of the routed queries.  Its answers must equal the GPU set's for the same keys."""
    from oracle import oqf

    qs, off, keys, qkeys = b["qs"], b["off"], b["keys"], b["qkeys"]
    threads = host_threads()
    stride = max(1, -(-int(off[-1]) // budget_keys))
    sample = list(range(0, nf, stride))
    shards = shard(sample, lambda i: int(off[i + 1] - off[i]), threads)
    fs, ans = {}, {}

    def qidx(i):
        return order[int(qoff[i]):int(qoff[i + 1])]

    def fill(sh):
        for i in sh:
            o = oqf.OracleQF(int(qs[i]), 8)
            assert o.insert(keys[int(off[i]):int(off[i + 1])]) == 0
            fs[i] = o

    def query(sh):
        for i in sh:
            ans[i] = fs[i].query(qkeys[qidx(i)])

    t_fill = pool_time(fill, shards, threads)
    t_query = pool_time(query, shards, threads)
    for i in sample:
        assert np.array_equal(ans[i], got_set[qidx(i)]), f"filter {i}: oracle and GPU answers differ"
    n_fill = int(sum(int(off[i + 1] - off[i]) for i in sample))
    n_query = int(sum(len(qidx(i)) for i in sample))
    del fs
    return {"value": round(n_fill / t_fill / 1e9, 6), "unit": "B inserts/s", "cores": threads, "kind": "oracle",
            "query_Bps": round(n_query / t_query / 1e9, 6),
            "sample": (f"oracle/oqf.c on every {stride}-th filter ({len(sample)} filters of q {int(min(qs[sample]))}"
                       f"..{int(max(qs[sample]))}, {n_fill} fill keys in one batch each, then their {n_query} routed "
                       f"queries), filters spread over {threads} threads; answers equal the GPU set's"),
            "host": host_cpu()}


def cpu_baseline_serve(qs, rs, fill, reqs, qmax: int = 20) -> dict:
    """The CPU oracle (oracle/oqf.c as it stands) serving the same request stream restricted to the
    filters of at most 2^qmax quotients, filters spread over all host threads (each thread replays
    its filters' requests in submission order).  The filters are filled beforehand (not timed)."""
    from oracle import oqf

    threads = host_threads()
    sample = [i for i in range(len(qs)) if int(qs[i]) <= qmax]
    mine = {i: [] for i in sample}
    for op, f, keys in reqs:
        if f in mine:
            mine[f].append((op, keys))
    shards = shard(sample, lambda i: sum(len(k) for _, k in mine[i]) + (1 << int(qs[i])) // 8, threads)
    fs = {}

    def build(sh):
        for i in sh:
            o = oqf.OracleQF(int(qs[i]), int(rs[i]))
            assert o.insert(fill[i]) == 0
            fs[i] = o

    def serve(sh):
        from paper_2212_09005_amd import qf

        for i in sh:
            o = fs[i]
            for op, keys in mine[i]:
                if op == qf.QFS_INSERT:
                    assert o.insert(keys) == 0
                elif op == qf.QFS_DELETE:
                    assert o.delete(keys)[0] == 0
                else:
                    o.query(keys)

    pool_time(build, shards, threads)
    dt = pool_time(serve, shards, threads)
    nreq = sum(len(v) for v in mine.values())
    nkeys = sum(len(k) for v in mine.values() for _, k in v)
    del fs
    return {"value": round(nkeys / dt / 1e9, 6), "unit": "B keys/s", "cores": threads, "kind": "oracle",
            "req_per_s": round(nreq / dt, 1),
            "sample": (f"oracle/oqf.c serving the saturation stream's {nreq} requests ({nkeys} keys) to the "
                       f"{len(sample)} filters of q <= {qmax}, filled beforehand (not timed), filters spread over "
                       f"{threads} threads, each filter's requests in order"),
            "host": host_cpu()}


def copy_bandwidth(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Attainable HBM bandwidth: a device-to-device copy of nbytes (read + write), GB/s, best of reps."""
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 0.0
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best = max(best, 2 * nbytes / (a.elapsed_time(b) * 1e-3) / 1e9)
    del src, dst
    return round(best, 1)


def bench_sets(args) -> dict:
    """Many filters (4096, 2^10..2^20 quotients, r = 8): fill each to load 0.85, then query 2^24 keys
    spread over the filters in proportion to their size (half present, half absent).  The same work
    runs three ways on the same GPU: a filter set with autotuned launch parameters whose fill and
    query are each one captured graph (the reported value), a filter set with default parameters
    called directly, and a plain loop of per-filter calls; answers and tables must come out
    identical."""
    import torch

    from paper_2212_09005_amd import inputs, qf

    from paper_2212_09005_amd.workloads import ManyFilters

    wl = ManyFilters(nf=args.sets_filters, query_log2=args.sets_query_log2)
    b = wl.build()
    nf, qs, fill_n, off, keys, fid = wl.nf, b["qs"], b["fill_n"], b["off"], b["keys"], b["fid"]
    total = int(off[-1])
    log(f"c4: {nf} filters, {total} fill keys, {int(sum(1 << int(q) for q in qs))} quotients")
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    d_fid = torch.from_numpy(fid).to("cuda")
    m = 1 << args.sets_query_log2
    qfid, qkeys, present, rng = b["qfid"], b["qkeys"], b["present"], b["rng"]
    d_qkeys = torch.from_numpy(qkeys.view(np.int64)).to("cuda")
    d_qfid = torch.from_numpy(qfid).to("cuda")
    # the per-filter loop gets its queries already grouped by filter (untimed)
    order = np.argsort(qfid, kind="stable")
    qoff = np.concatenate([[0], np.cumsum(np.bincount(qfid, minlength=nf))])
    d_qkeys_grouped = torch.from_numpy(qkeys[order].view(np.int64)).to("cuda")
    torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    sample = sorted(set(rng.integers(0, nf, size=8).tolist()) | {int(np.argmax(qs)), int(np.argmin(qs))})
    # the set with autotuned launch parameters, fill and query each captured
    # as one graph (the graph's launch is what is timed)
    t0 = time.perf_counter()
    tuning, tune_ms = qf.autotune_set([int(q) for q in qs], 8, 0.85, m)
    t_tune = time.perf_counter() - t0
    log(f"c4 autotune: {tuning} in {t_tune:.1f}s (sample insert {tune_ms[0]:.2f} ms, query {tune_ms[1]:.3f} ms)")
    fs_g = [qf.CQF(int(q), 8) for q in qs]
    st_g = qf.CQFSet(fs_g)
    st_g.tune(**tuning)
    st_g.reserve(total)
    gs = torch.cuda.Stream()
    out_g = torch.empty(m, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    g_fill, g_query = qf.Graph(gs), qf.Graph(gs)
    with g_fill:
        st_g.insert(d_fid, d_keys, stream=gs.cuda_stream)
    with g_query:
        st_g.query(d_qfid, d_qkeys, out_g, stream=gs.cuda_stream)
    t_g_fill = timed(lambda: g_fill.launch())
    assert st_g.sync() == 0
    g_query.launch()  # warm-up
    t_g_query = timed(lambda: g_query.launch())
    got_g = out_g.cpu().numpy()
    lay_g = {i: fs_g[i].export() for i in sample}
    g_fill.close()
    g_query.close()
    st_g.close()
    for f in fs_g:
        f.close()
    del fs_g, st_g
    log(f"c4 tuned set, graphs: fill {t_g_fill:.3f}s, query {t_g_query * 1e3:.2f} ms")
    # the set (scratch reserved beforehand, so no allocation is timed)
    fs_set = [qf.CQF(int(q), 8) for q in qs]
    st = qf.CQFSet(fs_set)
    st.reserve(total)
    t_set_fill = timed(lambda: st.insert(d_fid, d_keys))
    assert st.sync() == 0
    out_set = torch.empty(m, dtype=torch.uint8, device="cuda")
    st.query(d_qfid, d_qkeys, out_set)  # warm-up
    t_set_query = timed(lambda: st.query(d_qfid, d_qkeys, out_set))
    got_set = out_set.cpu().numpy()
    lay_set = {i: fs_set[i].export() for i in sample}
    st.close()
    for f in fs_set:
        f.close()
    del fs_set, st
    log(f"c4 set: fill {t_set_fill:.3f}s, query {t_set_query * 1e3:.2f} ms")
    # the loop of per-filter calls (scratch reserved beforehand)
    fs_loop = [qf.CQF(int(q), 8) for q in qs]
    for i, f in enumerate(fs_loop):
        f.reserve(int(fill_n[i]))

    def loop_fill():
        for i, f in enumerate(fs_loop):
            f.insert(d_keys[int(off[i]):int(off[i + 1])])

    t_loop_fill = timed(loop_fill)
    out_loop = torch.empty(m, dtype=torch.uint8, device="cuda")

    def loop_query():
        for i, f in enumerate(fs_loop):
            a, b = int(qoff[i]), int(qoff[i + 1])
            if b > a:
                f.query(d_qkeys_grouped[a:b], out_loop[a:b])

    loop_query()  # warm-up
    t_loop_query = timed(loop_query)
    for f in fs_loop:
        assert f.sync() == 0
    log(f"c4 loop: fill {t_loop_fill:.3f}s, query {t_loop_query * 1e3:.2f} ms")
    # same answers, same tables (a sample of filters, every size)
    got_loop = np.empty(m, np.uint8)
    got_loop[order] = out_loop.cpu().numpy()
    assert np.array_equal(got_set, got_loop), "set and loop answers differ"
    assert np.array_equal(got_g, got_loop), "tuned graph and loop answers differ"
    assert got_set[present].all(), "a present key was not found"
    for i in sample:
        rc1, l1 = lay_set[i]
        rc2, l2 = fs_loop[i].export()
        rc3, l3 = lay_g[i]
        assert rc1 == 0 and rc2 == 0 and rc3 == 0
        for name in ("occ_words", "runend_words", "slots", "offsets", "header"):
            assert np.array_equal(getattr(l1, name), getattr(l2, name)), f"filter {i}: {name} differs"
            assert np.array_equal(getattr(l3, name), getattr(l2, name)), f"filter {i}: {name} differs (graph)"
    fp_rate = float(got_set[~present].mean())
    for f in fs_loop:
        f.close()
    cpu = None
    if not args.no_cpu_baseline:
        log("c4: timing the CPU oracle on a sample of the filters, all host threads")
        cpu = cpu_baseline_sets(b, nf, order, qoff, got_set)
        log(f"c4 oracle: {cpu}")
    res = {
        "metric": "filter-set fill and query throughput (4096 filters of 2^10..2^20 quotients, r=8, load 0.85)",
        "value": round(total / t_g_fill / 1e9, 4),
        "unit": "B inserts/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wl.name(), "filters": nf, "fill_keys": total,
                   "queries": m},
        "tuned_graph": {"fill_s": round(t_g_fill, 4), "fill_Bps": round(total / t_g_fill / 1e9, 4),
                        "query_ms": round(t_g_query * 1e3, 3), "query_Bps": round(m / t_g_query / 1e9, 4),
                        "tuning": tuning, "autotune_s": round(t_tune, 2)},
        "set": {"fill_s": round(t_set_fill, 4), "fill_Bps": round(total / t_set_fill / 1e9, 4),
                "query_ms": round(t_set_query * 1e3, 3), "query_Bps": round(m / t_set_query / 1e9, 4)},
        "loop": {"fill_s": round(t_loop_fill, 4), "fill_Bps": round(total / t_loop_fill / 1e9, 4),
                 "query_ms": round(t_loop_query * 1e3, 3), "query_Bps": round(m / t_loop_query / 1e9, 4)},
        "speedup": {"fill": round(t_loop_fill / t_set_fill, 2), "query": round(t_loop_query / t_set_query, 2),
                    "tuned_graph_fill": round(t_loop_fill / t_g_fill, 2),
                    "tuned_graph_query": round(t_loop_query / t_g_query, 2)},
        "absent_positive_rate": round(fp_rate, 6),
        "cpu_baseline": cpu,
    }
    return res


def bench_sweep(args) -> dict:
    """Load sweep (2^28 quotients, r = 8): fill in batches of 2^22 keys to load 0.95; the batch that
    crosses each 0.05 step is split so the steps are exact.  After each step one query batch of 2^22
    keys (half present, half absent).  Insert rate per step = keys of the step / time of its batches."""
    import torch

    from paper_2212_09005_amd import inputs, qf

    q, r, m = args.q, 8, 1 << args.batch_log2
    N = 1 << q
    top = int(0.95 * N)
    keys = inputs.uniform_keys(1, top)
    f = qf.CQF(q, r)
    f.reserve(m)
    qout = torch.empty(m, dtype=torch.uint8, device="cuda")
    steps = []
    done = 0
    for k in range(1, 20):
        target = int(round(0.05 * k * N)) if k < 19 else top
        target = min(target, top)
        n_step = target - done
        d = torch.from_numpy(keys[done:target].view(np.int64)).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a in range(0, n_step, m):
            f.insert(d[a:a + m])
        torch.cuda.synchronize()
        t_ins = time.perf_counter() - t0
        assert f.sync() == 0
        done = target
        qk = inputs.mixed_queries(2000 + k, keys[:done], m // 2, m - m // 2)
        dq = torch.from_numpy(qk.view(np.int64)).to("cuda")
        f.query(dq, qout)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.query(dq, qout)
        torch.cuda.synchronize()
        t_q = time.perf_counter() - t0
        steps.append({"load": round(done / N, 4), "insert_Bps": round(n_step / t_ins / 1e9, 4),
                      "query_Bps": round(m / t_q / 1e9, 4)})
        log(f"sweep load {done / N:.2f}: insert {n_step / t_ins / 1e9:.3f} B/s, query {m / t_q / 1e9:.3f} B/s")
        del d, dq
    f.close()
    at9 = next(s_ for s_ in steps if abs(s_["load"] - 0.9) < 1e-3)
    return {"metric": METRIC + " (load sweep)", "value": at9["insert_Bps"], "unit": "B inserts/s at load 0.9",
            "n_gpus": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"cqf_q{q}_r8_sweep_to_0.95_batch{m}", "q": q, "r": r, "batch": m},
            "steps": steps}


def bench_zipf(args) -> dict:
    """Counting with skew (2^30 quotients, r = 16): insert 0.9 * 2^30 Zipf(1.1) instances over 2^28
    distinct values as one batch, count 2^26 keys uniform over the 2^28 values, then delete a
    random 25 % of the inserted instances.  --zipf-scale shrinks every size by 2^-scale."""
    import torch

    from paper_2212_09005_amd import inputs, qf

    from paper_2212_09005_amd.workloads import Counting

    sc = args.zipf_scale
    wl = Counting(q=30 - sc, universe_log2=28 - sc, count_log2=26 - sc)
    q, r, n, universe = wl.q, wl.r, wl.n, wl.universe
    t0 = time.time()
    keys = inputs.rank_to_key(wl.ranks())
    log(f"zipf: {n} instances generated in {time.time() - t0:.1f}s")
    f = qf.CQF(q, r)
    f.reserve(n)
    d = torch.from_numpy(keys.view(np.int64)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.insert(d)
    torch.cuda.synchronize()
    t_ins = time.perf_counter() - t0
    rc = f.sync()
    assert rc == 0, f"insert failed {rc}"
    ck = inputs.rank_to_key(wl.count_ranks())
    mc = len(ck)
    dc = torch.from_numpy(ck.view(np.int64)).to("cuda")
    cout = torch.empty(mc, dtype=torch.int64, device="cuda")
    f.count(dc, cout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.count(dc, cout)
    torch.cuda.synchronize()
    t_cnt = time.perf_counter() - t0
    dk = keys[wl.delete_mask()]
    ddel = torch.from_numpy(dk.view(np.int64)).to("cuda")
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.delete(ddel, nf)
    torch.cuda.synchronize()
    t_del = time.perf_counter() - t0
    assert f.sync() == 0 and int(nf.item()) == 0
    info = f.info()
    f.close()
    return {"metric": "counting insert / count / delete throughput with Zipf(1.1) keys", "value": round(n / t_ins / 1e9, 4),
            "unit": "B inserts/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": wl.name(), "q": q, "r": r,
                       "instances": n, "count_keys": mc, "delete_instances": int(len(dk))},
            "insert_Bps": round(n / t_ins / 1e9, 4), "count_Bps": round(mc / t_cnt / 1e9, 4),
            "delete_Bps": round(len(dk) / t_del / 1e9, 4), "device_bytes": info["device_bytes"]}


def bench_fill(args) -> dict:
    """One big batch (the paper's bulk set-up): insert 0.9 * 2^q distinct uniform keys into an empty
    filter (2^28 quotients, r = 8) as one batch, then query 2^22 keys (half present, half absent)."""
    import torch

    from paper_2212_09005_amd import inputs, qf

    q, r = args.q, 8
    n = int(0.9 * (1 << q))
    keys = inputs.uniform_keys(1, n)
    f = qf.CQF(q, r)
    f.reserve(n)
    d = torch.from_numpy(keys.view(np.int64)).to("cuda")
    times = []
    for rep in range(2):  # the second run on a fresh filter is the one reported
        if rep:
            f.close()
            f = qf.CQF(q, r)
            f.reserve(n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.insert(d)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        assert f.sync() == 0
    m = 1 << 22
    qk = inputs.mixed_queries(2000, keys, m // 2, m - m // 2)
    dq = torch.from_numpy(qk.view(np.int64)).to("cuda")
    out = torch.empty(m, dtype=torch.uint8, device="cuda")
    f.query(dq, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.query(dq, out)
    torch.cuda.synchronize()
    tq = time.perf_counter() - t0
    f.close()
    return {"metric": "one-batch bulk insert (empty to load 0.9), then query", "value": round(n / times[-1] / 1e9, 4),
            "unit": "B inserts/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"cqf_q{q}_r8_one_batch_fill_0.9", "q": q, "r": r, "keys": n},
            "insert_s": round(times[-1], 4), "query_Bps": round(m / tq / 1e9, 4)}


def bench_point(args) -> dict:
    """Point updates of the counting quotient filter (qf_point_insert / qf_point_delete, one
    lane per key in place under region locks) at 2^q quotients, r = 8: fill an empty filter
    to load 0.9 with calls of 2^23 keys, then delete the first 2^23 keys with one point call.
    The table afterwards must hold exactly what a bulk insert of the same keys gives (stats)."""
    import torch

    from paper_2212_09005_amd import inputs, qf

    q, r = args.q, 8
    n = int(0.9 * (1 << q))
    chunk = 1 << 23
    f = qf.CQF(q, r)
    warm = torch.from_numpy(inputs.uniform_keys(3, 1 << 16).view(np.int64)).to("cuda")
    f.point_insert(warm)
    f.point_delete(warm)
    assert f.sync() == 0
    t_all, rates = 0.0, []
    first = None
    for lo in range(0, n, chunk):
        k = inputs.uniform_keys(100 + lo // chunk, min(chunk, n - lo))
        d = torch.from_numpy(k.view(np.int64)).to("cuda")
        if first is None:
            first = d
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.point_insert(d)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_all += dt
        rates.append((round(f.stats()["used"] / (1 << q), 3), round(len(k) / dt / 1e6, 1)))
    assert f.sync() == 0
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.point_delete(first, not_found=nf)
    torch.cuda.synchronize()
    t_del = time.perf_counter() - t0
    assert f.sync() == 0 and int(nf.item()) == 0
    f.close()
    return {"metric": "point inserts (one lane per key, region locks) from empty to load 0.9",
            "value": round(n / t_all / 1e6, 1), "unit": "M inserts/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"cqf_q{q}_r8_point_fill_0.9", "q": q, "r": r, "keys": n, "call_keys": chunk},
            "by_fill_Mps": rates[::4] + [rates[-1]], "delete_Mps": round(chunk / t_del / 1e6, 1)}


def bench_tcf(args) -> dict:
    """The two-choice filter at 2^28 slots (the size of the paper's CPU/GPU table, Sec. 6):
    point form (16-tag blocks) filled to load 0.9 by 2^24-key point calls, then 2^24 positive
    and 2^24 random (absent) lookups and 2^24 deletes; bulk form (128-tag sorted blocks) filled
    to load 0.9 by one batch and, on a second filter, by batches of 2^22 keys, then the same
    lookups.  Every present key must be found."""
    import torch

    from paper_2212_09005_amd import inputs, tcf

    slots = 1 << 28
    n = int(0.9 * slots)
    m = 1 << 24

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to("cuda")

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    keys = inputs.uniform_keys(1, n)
    d = dev(keys)
    absent = dev(inputs.absent_keys(2, m))
    pos = dev(keys[:m])
    out = torch.empty(m, dtype=torch.uint8, device="cuda")
    res = {}
    # point form
    t = tcf.TCF(slots // 16, tcf.TCF_POINT)
    warm = dev(inputs.uniform_keys(3, 1 << 16))
    t.insert(warm)
    t.delete(warm)
    ti = sum(timed(lambda lo=lo: t.insert(d[lo:lo + m])) for lo in range(0, n, m))
    assert t.sync() == 0
    tq = timed(lambda: t.query(pos, out))
    assert bool(out.all().item()), "point TCF: a present key was not found"
    tr = timed(lambda: t.query(absent, out))
    fp = int(out.sum().item())
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    td = timed(lambda: t.delete(pos, not_found=nf))
    info = t.info()
    res["point"] = {"insert_Bps": round(n / ti / 1e9, 3), "query_pos_Bps": round(m / tq / 1e9, 3),
                    "query_rand_Bps": round(m / tr / 1e9, 3), "delete_Bps": round(m / td / 1e9, 3),
                    "false_pos_rate": round(fp / m, 6), "backing_fraction": round(info["backing_used"] / n, 6),
                    "deletes_not_found": int(nf.item())}
    t.close()
    # bulk form, one batch
    t = tcf.TCF(slots // 128, tcf.TCF_BULK)
    t.insert(warm)
    t.delete(warm)
    ti = timed(lambda: t.insert(d))
    tq = timed(lambda: t.query(pos, out))
    assert bool(out.all().item()), "bulk TCF: a present key was not found"
    tr = timed(lambda: t.query(absent, out))
    fp = int(out.sum().item())
    td = timed(lambda: t.delete(pos[: 1 << 22]))
    res["bulk_one_batch"] = {"insert_Bps": round(n / ti / 1e9, 3), "query_pos_Bps": round(m / tq / 1e9, 3),
                             "query_rand_Bps": round(m / tr / 1e9, 3),
                             "delete_2p22_Bps": round((1 << 22) / td / 1e9, 3), "false_pos_rate": round(fp / m, 6)}
    t.close()
    # bulk form, batches of 2^22
    t = tcf.TCF(slots // 128, tcf.TCF_BULK)
    b = 1 << 22
    ti = sum(timed(lambda lo=lo: t.insert(d[lo:lo + b])) for lo in range(0, n, b))
    res["bulk_batches_2p22"] = {"insert_Bps": round(n / ti / 1e9, 3)}
    t.close()
    return {"metric": "two-choice filter at 2^28 slots: point and bulk insert / lookup rates",
            "value": res["point"]["insert_Bps"], "unit": "B point inserts/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "tcf_2p28_slots_load_0.9", "slots": slots, "keys": n, "lookups": m},
            **res}


def bench_serve(args) -> dict:
    """Serving: 256 device-resident filters (2^18..2^26 quotients, r = 8 or 16), filled to load 0.5,
    answer Poisson arrivals of mixed requests (70 % query, 25 % insert, 5 % delete) with sizes
    log-uniform in 1..65,536 keys, HBM budget 64 GB.  A saturation run measures capacity (and the
    same request stream replayed as a plain loop of per-request calls gives the baseline); then
    arrivals at 25 / 50 / 90 % of it give ops/s and p50 / p99 latency (submission to completion)."""
    import threading

    from paper_2212_09005_amd import inputs, qf

    from paper_2212_09005_amd.workloads import Serving

    wl = Serving(nf=args.serve_filters)
    nf = wl.nf
    qs, rs = wl.filters()
    srv = qf.Server(64 << 30, max_round_keys=1 << 22)
    ids = [srv.open(int(q), int(r)) for q, r in zip(qs, rs)]
    fill = wl.fill_keys(qs)
    tag = 0
    for i, k in enumerate(fill):
        for a in range(0, len(k), 1 << 22):
            srv.submit(qf.QFS_INSERT, ids[i], k[a:a + (1 << 22)], tag)
            tag += 1
    got = 0
    while got < tag:
        got += len(srv.poll(4096, 100000))
    log(f"serve: {nf} filters filled to {wl.load0} ({sum(len(k) for k in fill)} keys)")
    # per-filter key counts and delete cursors, carried across the request streams
    state = {"count": np.array([len(k) for k in fill], dtype=np.int64), "dcur": np.zeros(nf, np.int64)}

    def make_requests(nreq, seed):
        return wl.requests(nreq, seed, qs, fill, state)

    def run(reqs, rate):
        """Submit reqs with Poisson arrivals at `rate` requests/s (None = as fast as possible)."""
        nonlocal tag
        sub = {}
        lat = []
        done = threading.Event()
        base_tag = tag

        def poller():
            left = len(reqs)
            while left:
                for t, st in srv.poll(4096, 2000):
                    lat.append(time.perf_counter() - sub[t])
                    left -= 1
            done.set()

        th = threading.Thread(target=poller)
        g = np.random.Generator(np.random.PCG64(99))
        gaps = g.exponential(1.0 / rate, size=len(reqs)) if rate else np.zeros(len(reqs))
        t_start = time.perf_counter()
        t_next = t_start
        th.start()
        for k, (op, f, keys) in enumerate(reqs):
            t_next += gaps[k]
            while rate and time.perf_counter() < t_next:
                pass
            t = base_tag + k
            sub[t] = time.perf_counter()
            srv.submit(op, ids[f], keys, t)
        done.wait()
        th.join()
        t_end = time.perf_counter()
        tag = base_tag + len(reqs)
        nkeys = sum(len(k) for _, _, k in reqs)
        lat_ms = np.array(lat) * 1e3
        return {"requests": len(reqs), "keys": nkeys, "seconds": round(t_end - t_start, 4),
                "Bps": round(nkeys / (t_end - t_start) / 1e9, 4),
                "req_per_s": round(len(reqs) / (t_end - t_start), 1),
                "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 3)}

    nreq = args.serve_requests
    sat_reqs = make_requests(nreq, 1)
    st0 = srv.stats()
    sat = run(sat_reqs, None)
    st1 = srv.stats()
    sat["server"] = {k: st1[k] - st0[k] for k in ("rounds", "requests", "keys", "updates_in_place", "updates_bulk",
                                                  "ns_form", "ns_launch", "ns_wait", "ns_complete", "ns_stage")}
    log(f"serve saturation: {sat}")
    loop = loop_replay(qs, rs, fill, sat_reqs, qf)
    log(f"serve, same stream as a loop of per-request calls: {loop}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_serve(qs, rs, fill, sat_reqs)
        log(f"serve oracle: {cpu}")
    cap_rps = sat["req_per_s"]
    points = []
    for frac in (0.25, 0.5, 0.9):
        r_ = run(make_requests(nreq, 2 + int(frac * 100)), frac * cap_rps)
        r_["offered_frac"] = frac
        points.append(r_)
        log(f"serve at {frac:.0%} of capacity: {r_}")
    st = srv.stats()
    srv.close()
    sat["vs_loop"] = round(sat["Bps"] / loop["Bps"], 2)
    return {"metric": "serving: mixed request throughput and latency (256 filters, 2^18..2^26, r=8/16)",
            "value": sat["Bps"], "unit": "B keys/s at saturation", "n_gpus": 1, "higher_is_better": True,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": wl.name(), "filters": nf,
                       "requests_per_run": nreq, "budget_bytes": 64 << 30},
            "saturation": sat, "loop": loop, "points": points, "server": st, "cpu_baseline": cpu}


def loop_replay(qs, rs, fill, reqs, qf) -> dict:
    """The plain per-filter launch loop: filters of the same sizes and contents, and the same request
    stream as direct calls in submission order (keys copied to the device per request, query
    answers copied back per request, as the server does)."""
    import torch

    fs = [qf.CQF(int(q), int(r)) for q, r in zip(qs, rs)]
    dbuf = torch.empty(1 << 22, dtype=torch.int64, device="cuda")
    for i, k in enumerate(fill):
        for a in range(0, len(k), 1 << 22):
            part = k[a:a + (1 << 22)]
            dbuf[:len(part)].copy_(torch.from_numpy(part.view(np.int64)))
            fs[i].insert(dbuf[:len(part)])
    for f in fs:
        f.reserve(1 << 16)
    nf_buf = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op, f, keys in reqs:
        d = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).to("cuda")
        if op == qf.QFS_INSERT:
            fs[f].insert(d)
        elif op == qf.QFS_DELETE:
            fs[f].delete(d, nf_buf)
        else:
            fs[f].query(d).cpu()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for f in fs:
        assert f.sync() == 0
        f.close()
    nkeys = sum(len(k) for _, _, k in reqs)
    return {"requests": len(reqs), "keys": nkeys, "seconds": round(dt, 4), "Bps": round(nkeys / dt / 1e9, 4),
            "req_per_s": round(len(reqs) / dt, 1)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--q", type=int, default=28)
    ap.add_argument("--load", type=float, default=0.9)
    ap.add_argument("--batch-log2", type=int, default=22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["c2", "sweep", "fill", "zipf", "c4", "serve", "tcf", "point"],
                    default="c2",
                    help="c2: the single-filter step (default); sweep: load sweep to 0.95; fill: one-batch fill "
                         "to 0.9; zipf: one-batch counting with skew (2^30, r=16); c4: many filters, set vs "
                         "per-filter loop; serve: the serving loop; tcf: the two-choice filter at 2^28 slots; point: "
                         "point inserts of the counting filter to load 0.9")
    ap.add_argument("--serve-filters", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=4000)
    ap.add_argument("--zipf-scale", type=int, default=0)
    ap.add_argument("--sets-filters", type=int, default=4096)
    ap.add_argument("--sets-query-log2", type=int, default=24)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB before the fill, as the "
                         "reference kernel for HBM byte counters (FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the filter's multi-GPU sharding is a "
              f"design note, not a benchmark here.", file=sys.stderr)
        return 2

    import torch

    from paper_2212_09005_amd import qf
    from paper_2212_09005_amd.workloads import LoadSweep

    if args.workload != "c2":
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        torch.cuda.set_device(0)
        fn = {"c4": bench_sets, "sweep": bench_sweep, "fill": bench_fill, "zipf": bench_zipf,
              "serve": bench_serve, "tcf": bench_tcf, "point": bench_point}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return 0

    w = LoadSweep(q=args.q, load=args.load, batch=1 << args.batch_log2)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {nb} bytes device to device (counter calibration)")
        del src, dst
    log(f"workload: {w.name()}")

    t0 = time.time()
    fill = w.fill_keys()
    log(f"generated {len(fill)} fill keys in {time.time() - t0:.1f}s")
    f = qf.CQF(w.q, w.r)
    d_batch = torch.empty(w.batch, dtype=torch.int64, device="cuda")
    for i, s in enumerate(range(0, len(fill), w.batch)):
        part = fill[s : s + w.batch]
        d = d_batch[: len(part)]
        d.copy_(torch.from_numpy(part.view(np.int64)))
        f.insert(d)
        if i % 16 == 0:
            torch.cuda.synchronize()
            log(f"fill batch {i}: {s + len(part)} keys")
    torch.cuda.synchronize()
    assert f.sync() == 0, "fill failed"
    log(f"filled to load {w.load} in {time.time() - t0:.1f}s")

    nsteps = args.warmup + args.steps
    ins = [to_dev(w.insert_keys(i), torch) for i in range(nsteps)]
    qry = [to_dev(w.query_keys(i, fill), torch) for i in range(nsteps)]
    qout = torch.empty(w.batch, dtype=torch.uint8, device="cuda")
    cout = torch.empty(w.batch, dtype=torch.int64, device="cuda")
    nf = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    def step(i, ev=None):
        if ev is not None:
            ev[0].record()
        f.insert(ins[i])
        if ev is not None:
            ev[1].record()
        f.query(qry[i], qout)
        if ev is not None:
            ev[2].record()
        f.count(qry[i], cout)
        if ev is not None:
            ev[3].record()
        f.delete(ins[i], nf)
        if ev is not None:
            ev[4].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    assert f.sync() == 0
    log("warmup done")

    # The timed region: HIP events on the launch stream bracket only the merge
    # launches (the roofline kernel); every event pair holds the stream for a
    # few microseconds, so the other kernels run unbracketed.
    # Events recorded on the stream between the operations of each step give
    # the per-operation rates (insert and query are the metric's two numbers)
    # from the timed steps themselves.
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    qf.qf_profile_enable(f.h, True, kinds=("merge",))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, events[k])
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    prof_timed = qf.qf_profile_read(f.h)
    qf.qf_profile_enable(f.h, False)
    rc = f.sync()
    assert rc == 0, f"deferred error {rc}"
    elapsed = t_end - t_start
    op_ms = np.zeros(4)
    for ev in events:
        for j in range(4):
            op_ms[j] += ev[j].elapsed_time(ev[j + 1])
    op_ms /= args.steps
    # An untimed replay of the same steps (each step leaves the table as it
    # found it) with every kernel kind bracketed: the kernel breakdown.
    qf.qf_profile_enable(f.h, True)
    for k in range(args.steps):
        step(args.warmup + k)
    torch.cuda.synchronize()
    prof = qf.qf_profile_read(f.h)
    qf.qf_profile_enable(f.h, False)
    assert f.sync() == 0
    # sanity on the last step's outputs: present keys are found, deletes all hit
    assert int(nf.item()) == 0, "a delete missed"
    log(f"timed {args.steps} steps in {elapsed * 1e3:.1f} ms")

    m = w.batch
    total_ops = 4.0 * m * args.steps
    consts = load_constants(w)
    kinds = {}
    for kind, (ms, n) in prof.items():
        if n == 0:
            continue
        per = ms / n
        ab = algorithmic_bytes(kind, w, consts, 0.5)
        kinds[kind] = {"ms_total": round(ms, 4), "launches": n, "ms_per_launch": round(per, 5)}
        if ab is not None:
            gbs = ab / (per * 1e-3) / 1e9
            kinds[kind].update({"alg_bytes_per_launch": ab, "alg_GBs": round(gbs, 1),
                                "frac": round(gbs / HBM_PEAK_GBS, 4)})
    dom = max(kinds, key=lambda k: kinds[k]["ms_total"])
    timed = {k: v for k, v in kinds.items() if "alg_GBs" in v}
    rk = dom if dom in timed else max(timed, key=lambda k: timed[k]["ms_total"]) if timed else None
    roofline = None
    if rk is not None and prof_timed[rk][1] > 0:
        # the roofline kernel's launches inside the timed region
        ms_t, n_t = prof_timed[rk]
        per_t = ms_t / n_t
        gbs = algorithmic_bytes(rk, w, consts, 0.5) / (per_t * 1e-3) / 1e9
        traffic = (measured_traffic("k_" + rk) if (w.q, w.r, w.load, w.batch) == (28, 8, 0.9, 1 << 22) else None)
        roofline = {"kernel": rk, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "ms_per_launch": round(per_t, 5), "launches": n_t,
                    "time_share": round(ms_t / (elapsed * 1e3), 3)}
    # whole operations against the same roofline: algorithmic bytes per key
    # (the key in, the grouping round trip of an update, the changed blocks
    # read and written, the distinct blocks a lookup reads, the result out)
    op_roof = None
    if consts is not None:
        Bb = 64 * (w.r + 2) // 8 + 1
        per_key = {"insert": 8.0 + 16.0 + 2.0 * Bb * consts["C_mean"] / m,
                   "query": 8.0 + 1.0 + Bb * consts["D_mean"] / m,
                   "count": 8.0 + 8.0 + Bb * consts["D_mean"] / m,
                   "delete": 8.0 + 16.0 + 2.0 * Bb * consts["C_mean"] / m}
        op_roof = {}
        for j, k in enumerate(("insert", "query", "count", "delete")):
            gbs = per_key[k] * m / (op_ms[j] * 1e-3) / 1e9
            op_roof[k] = {"alg_bytes_per_key": round(per_key[k], 2), "GBs": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4)}
    attainable = copy_bandwidth(torch)
    if roofline is not None:
        roofline["attainable_copy_GBs"] = attainable
    out = {
        "metric": METRIC,
        "value": round(total_ops / elapsed / 1e9, 4),
        "unit": "B ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name(), "q": w.q, "r": w.r, "load": w.load, "batch": m,
                   "ops_per_step": 4 * m},
        # the metric's two numbers, from the timed steps
        "insert_Bps": round(m / op_ms[0] / 1e6, 4),
        "query_Bps": round(m / op_ms[1] / 1e6, 4),
        "rates_Bps": {
            "insert": round(m / op_ms[0] / 1e6, 4),
            "query": round(m / op_ms[1] / 1e6, 4),
            "count": round(m / op_ms[2] / 1e6, 4),
            "delete": round(m / op_ms[3] / 1e6, 4),
        },
        "op_ms": {k: round(float(v), 4) for k, v in zip(("insert", "query", "count", "delete"), op_ms)},
        "op_roofline": op_roof,
        "attainable_copy_GBs": attainable,
        # every kind bracketed, in an untimed replay of the same steps
        "kernels": kinds,
        "dominant_kernel": dom,
        "roofline": roofline,
    }
    f.close()
    del ins, qry
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample of the same step")
        out["cpu_baseline"] = cpu_baseline(w, fill)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
