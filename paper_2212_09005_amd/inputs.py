"""Seeded synthetic key streams shared by the GPU tests, the bench and the oracle checks.

This module holds none of the filter's arithmetic (no hashing, no fingerprint
split): it only draws 64-bit keys from numpy's PCG64 generator.  Both the GPU
path and the CPU oracles receive the same arrays.

Recipes (the paper's micro-benchmarks hash random 64-bit words from a seeded
generator and draw the absent lookups from a second seed, Sec. 6 set-up; the
counting benchmark uses Zipfian counts, Sec. 6.7):
  * present keys: 63-bit uniform values (top bit 0) from PCG64(seed);
  * absent keys: 63-bit uniform values with the top bit set, from another seed,
    so they can never equal a present key;
  * Zipf keys: rank k in [1, universe] drawn with P(k) ~ k^-s by
    rejection-inversion (Hoermann and Derflinger 1996), then mapped to a key
    by an odd-multiplier bijection (distinct ranks give distinct keys).
"""
from __future__ import annotations

import numpy as np

U64 = np.uint64
_TOP = U64(1) << U64(63)
_LOW63 = _TOP - U64(1)


def _gen(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_keys(seed: int, n: int, distinct: bool = False) -> np.ndarray:
    """n present keys (top bit clear).  With distinct=True, repeats are dropped
    (first occurrence kept, order preserved) and the stream is extended."""
    g = _gen(seed)
    if not distinct:
        return g.integers(0, 1 << 63, size=n, dtype=np.uint64)
    out = np.zeros(0, dtype=U64)
    want = n
    while len(out) < n:
        more = g.integers(0, 1 << 63, size=want + 64, dtype=np.uint64)
        allk = np.concatenate([out, more])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        out = allk[first]
        want = n - len(out)
    return out[:n].copy()


def absent_keys(seed: int, n: int) -> np.ndarray:
    """n keys with the top bit set (never equal to a present key)."""
    g = _gen(seed)
    return g.integers(0, 1 << 63, size=n, dtype=np.uint64) | _TOP


def sample_without_replacement(seed: int, population: int, n: int) -> np.ndarray:
    """n distinct indices in [0, population), uniformly at random."""
    g = _gen(seed)
    return g.choice(population, size=n, replace=False).astype(np.int64)


def shuffle(seed: int, a: np.ndarray) -> np.ndarray:
    g = _gen(seed)
    return a[g.permutation(len(a))]


def mixed_queries(seed: int, present: np.ndarray, n_present: int, n_absent: int) -> np.ndarray:
    """n_present keys drawn without replacement from `present` plus n_absent
    absent keys, interleaved by a seeded shuffle."""
    idx = sample_without_replacement(seed, len(present), n_present)
    q = np.concatenate([present[idx], absent_keys(seed + 1_000_003, n_absent)])
    return shuffle(seed + 2_000_003, q)


_ZIPF_MUL = U64(0x9E3779B97F4A7C15)  # odd, so k -> k * M is a bijection mod 2^64


_ZIPF_CHUNK = 1 << 22


def _zipf_chunk(seed: int, j: int, n: int, s: float, universe: int) -> np.ndarray:
    """n Zipf ranks by rejection-inversion (Hoermann and Derflinger, ACM TOMACS
    1996): with h(x) = x^-s and its integral H, draw u uniformly from
    [H(3/2) - h(1), H(universe + 1/2)], invert it to x = H^-1(u), round to k and
    keep k when u lies in the top h(k) of k's share [H(k - 1/2), H(k + 1/2)]
    (so P(k) is exactly proportional to h(k); k = 1's share is h(1) long)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, j])))
    a = 1.0 - s

    def H(x):
        return np.expm1(a * np.log(x)) / a

    def Hinv(y):
        return np.exp(np.log1p(a * y) / a)

    lo = float(H(np.float64(1.5))) - 1.0
    hi = float(H(np.float64(universe + 0.5)))
    out = np.empty(n, dtype=np.int64)
    filled = 0
    while filled < n:
        need = n - filled
        u = hi + g.random(need + need // 16 + 64) * (lo - hi)
        x = Hinv(u)
        k = np.clip(np.floor(x + 0.5), 1, universe)
        ok = u >= H(k + 0.5) - np.exp(-s * np.log(k))
        k = k[ok][:need].astype(np.int64)
        out[filled:filled + len(k)] = k
        filled += len(k)
    return out


def zipf_ranks(seed: int, n: int, s: float = 1.1, universe: int = 1 << 28) -> np.ndarray:
    """n ranks in [1, universe] with P(k) proportional to k^-s (s > 0, s != 1).
    The stream is cut into chunks of 2^22 draws, chunk j from its own PCG64
    generator seeded by (seed, j); chunks are drawn on several threads and the
    result does not depend on how many."""
    import concurrent.futures as cf
    import os

    out = np.empty(n, dtype=np.int64)
    starts = list(range(0, n, _ZIPF_CHUNK))

    def work(j):
        a = starts[j]
        b = min(a + _ZIPF_CHUNK, n)
        out[a:b] = _zipf_chunk(seed, j, b - a, s, universe)

    with cf.ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        list(ex.map(work, range(len(starts))))
    return out


def rank_to_key(ranks: np.ndarray, salt: int = 0x5DEECE66D) -> np.ndarray:
    with np.errstate(over="ignore"):
        return (np.asarray(ranks, dtype=U64) * _ZIPF_MUL) ^ U64(salt)


def zipf_keys(seed: int, n: int, s: float = 1.1, universe: int = 1 << 28) -> np.ndarray:
    return rank_to_key(zipf_ranks(seed, n, s, universe))


def bernoulli_mask(seed: int, n: int, p: float) -> np.ndarray:
    return _gen(seed).random(n) < p
