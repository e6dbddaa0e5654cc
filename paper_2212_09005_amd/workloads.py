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
