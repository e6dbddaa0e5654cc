"""Benchmark workloads: sizes and seeded key streams (no filter arithmetic).

C2 ("load sweep"): one filter with 2^28 quotients and 8-bit remainders.
  * fill: floor(load * 2^28) uniform 63-bit keys (seed 1), inserted in
    batches of 2^22 -- the paper's micro-benchmark fills a filter with hashed
    random 64-bit items up to its recommended load (Sec. 6 set-up);
  * step i: insert 2^22 fresh uniform keys (seed 1000 + i), query 2^22 keys
    that are half present (drawn without replacement from the fill keys) and
    half absent (top bit set), count the same 2^22 keys, then delete the
    batch inserted in this step, so the table returns to the same load.
C1 ("small"): 2^16 quotients, r = 8, 58,982 distinct keys in one batch.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import inputs


@dataclass(frozen=True)
class LoadSweep:
    q: int = 28
    r: int = 8
    load: float = 0.9
    batch: int = 1 << 22
    fill_seed: int = 1

    @property
    def n_fill(self) -> int:
        return int(self.load * (1 << self.q))

    def fill_keys(self) -> np.ndarray:
        return inputs.uniform_keys(self.fill_seed, self.n_fill)

    def insert_keys(self, step: int) -> np.ndarray:
        return inputs.uniform_keys(1000 + step, self.batch)

    def query_keys(self, step: int, fill: np.ndarray) -> np.ndarray:
        half = self.batch // 2
        return inputs.mixed_queries(2000 + 10 * step, fill, half, self.batch - half)

    def name(self) -> str:
        return (f"cqf_q{self.q}_r{self.r}_load{self.load:g}_batch{self.batch}: insert + query(50% present) "
                f"+ count + delete of one batch")


C2 = LoadSweep()


# ---------------------------------------------------------------------------
# C3 ("counting with skew"): one filter with 2^30 quotients and 16-bit
# remainders; 0.9 * 2^30 instances drawn Zipf(1.1) over 2^28 distinct values
# inserted as one batch (the paper's counting runs insert the whole data set
# as one batch, Sec. 6.7); then counts of 2^26 keys uniform over the 2^28
# values (hot, cold and never-drawn ones) and the delete of a random 25 % of
# the inserted instances (each kept or dropped by a seeded coin).
@dataclass(frozen=True)
class Counting:
    q: int = 30
    r: int = 16
    s: float = 1.1
    universe_log2: int = 28
    seed: int = 3
    count_log2: int = 26
    count_seed: int = 4
    delete_frac: float = 0.25
    delete_seed: int = 5

    @property
    def n(self) -> int:
        return int(0.9 * (1 << self.q))

    @property
    def universe(self) -> int:
        return 1 << self.universe_log2

    def ranks(self) -> np.ndarray:
        return inputs.zipf_ranks(self.seed, self.n, self.s, self.universe)

    def count_ranks(self) -> np.ndarray:
        g = np.random.Generator(np.random.PCG64(self.count_seed))
        return g.integers(1, self.universe + 1, size=1 << self.count_log2)

    def delete_mask(self) -> np.ndarray:
        return inputs.bernoulli_mask(self.delete_seed, self.n, self.delete_frac)

    def name(self) -> str:
        return f"cqf_q{self.q}_r{self.r}_zipf{self.s:g}_universe2^{self.universe_log2}_one_batch"


# ---------------------------------------------------------------------------
# C4 ("many filters"): 4096 filters with q uniform in {10..20} (log-uniform
# sizes) and r = 8, each filled to load 0.85 by one batch of uniform keys
# tagged with filter indexes; then 2^24 queries whose filter is drawn in
# proportion to 2^q, half of them present keys of that filter, half absent.
@dataclass(frozen=True)
class ManyFilters:
    nf: int = 4096
    qlo: int = 10
    qhi: int = 20
    r: int = 8
    load: float = 0.85
    query_log2: int = 24
    seed: int = 5

    def build(self) -> dict:
        rng = np.random.Generator(np.random.PCG64(self.seed))
        qs = rng.integers(self.qlo, self.qhi + 1, size=self.nf)
        fill_n = np.array([int(self.load * (1 << int(q))) for q in qs], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(fill_n)])
        total = int(off[-1])
        keys = inputs.uniform_keys(self.seed, total)
        fid = np.repeat(np.arange(self.nf, dtype=np.int32), fill_n)
        m = 1 << self.query_log2
        w = np.array([2.0 ** int(q) for q in qs])
        qfid = rng.choice(self.nf, size=m, p=w / w.sum()).astype(np.int32)
        present = rng.random(m) < 0.5
        qkeys = inputs.absent_keys(self.seed + 1, m)
        pidx = off[qfid] + (rng.random(m) * fill_n[qfid]).astype(np.int64)
        qkeys[present] = keys[pidx[present]]
        return {"qs": qs, "fill_n": fill_n, "off": off, "keys": keys, "fid": fid, "qfid": qfid,
                "qkeys": qkeys, "present": present, "rng": rng}

    def name(self) -> str:
        return f"c4_sets_{self.nf}filters_q{self.qlo}to{self.qhi}_r{self.r}_load{self.load:g}"


# ---------------------------------------------------------------------------
# C5 ("serving"): 256 device-resident filters, q uniform in {18..26}, r = 8 or
# 16 (even odds), filled to load 0.5; requests are 70 % query, 25 % insert,
# 5 % delete, each on a uniformly drawn filter, with floor(2^U(0, 16)) keys
# (log-uniform in 1..65,536).  A query holds present keys of its filter and
# as many absent ones; an insert brings fresh keys (moved to another filter
# when it would take its filter past load 0.95); a delete removes fill keys
# of its filter, each fill key at most once over the stream, so a delete
# never asks for more copies than are stored.
@dataclass(frozen=True)
class Serving:
    nf: int = 256
    qlo: int = 18
    qhi: int = 26
    load0: float = 0.5
    cap: float = 0.95
    seed: int = 55
    max_log2: int = 16

    def filters(self) -> tuple[np.ndarray, np.ndarray]:
        rng = np.random.Generator(np.random.PCG64(self.seed))
        qs = rng.integers(self.qlo, self.qhi + 1, size=self.nf)
        rs = np.where(rng.random(self.nf) < 0.5, 8, 16)
        return qs, rs

    def fill_keys(self, qs) -> list:
        import concurrent.futures as cf
        import os

        def one(i):
            return inputs.uniform_keys(7000 + i, int(self.load0 * (1 << int(qs[i]))))

        with cf.ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
            return list(ex.map(one, range(len(qs))))

    def requests(self, nreq: int, seed: int, qs, fills, state: dict | None = None) -> list:
        """(op, filter, keys) with op 0 insert, 1 delete, 2 query (the server's QFS_* codes).  `state`
        (per-filter key counts and delete cursors) carries over between streams on the same filters."""
        g = np.random.Generator(np.random.PCG64(seed))
        nf = len(qs)
        if state is None:
            state = {"count": np.array([len(k) for k in fills], dtype=np.int64),
                     "dcur": np.zeros(nf, dtype=np.int64)}
        count, dcur = state["count"], state["dcur"]
        cap_keys = np.array([int(self.cap * (1 << int(q))) for q in qs])
        ops = g.choice(3, size=nreq, p=[0.70, 0.25, 0.05])
        sizes = np.floor(2.0 ** g.uniform(0, self.max_log2, size=nreq)).astype(np.int64)
        fids = g.integers(0, nf, size=nreq)
        reqs = []
        for k in range(nreq):
            f, n = int(fids[k]), int(sizes[k])
            op = int(ops[k])
            if op == 1:  # insert, moved when the filter would pass the cap
                if count[f] + n > cap_keys[f]:
                    room = np.nonzero(count + n <= cap_keys)[0]
                    if len(room) == 0:
                        op = 0
                    else:
                        f = int(room[g.integers(0, len(room))])
                if op == 1:
                    count[f] += n
                    reqs.append((0, f, inputs.uniform_keys(seed * 1_000_003 + k, n)))
                    continue
            if op == 2:  # delete fill keys not deleted before
                n = min(n, len(fills[f]) - int(dcur[f]))
                keys = fills[f][dcur[f]:dcur[f] + n]
                dcur[f] += n
                count[f] -= n
                reqs.append((1, f, keys))
                continue
            half = n // 2
            pres = fills[f][g.integers(0, len(fills[f]), size=n - half)]
            reqs.append((2, f, np.concatenate([pres, inputs.absent_keys(seed * 7 + k, half)])))
        return reqs

    def name(self) -> str:
        return f"serve_{self.nf}filters_q{self.qlo}to{self.qhi}_r8or16_mix70q25i5d"


C3 = Counting()
C4 = ManyFilters()
C5 = Serving()
