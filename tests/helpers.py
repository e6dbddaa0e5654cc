"""Test-only helpers: golden-file readers and key crafting.

Crafting keys with a chosen fingerprint needs the inverse of the SplitMix64
finalizer; it lives here (test code), not in the oracle or the library.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
M64 = (1 << 64) - 1
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB
_C1_INV = pow(_C1, -1, 1 << 64)
_C2_INV = pow(_C2, -1, 1 << 64)


def golden_lines(name: str):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def _unxorshift(y: np.ndarray, k: int) -> np.ndarray:
    x = y.copy()
    for _ in range(64 // k + 1):
        x = y ^ (x >> np.uint64(k))
    return x


def fin64_inverse(h: np.ndarray) -> np.ndarray:
    """Inverse of z -> SplitMix64 finalizer(z): undo each xorshift by
    iteration and each odd multiplier by its inverse mod 2^64."""
    z = np.asarray(h, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = _unxorshift(z, 31)
        z = z * np.uint64(_C2_INV)
        z = _unxorshift(z, 27)
        z = z * np.uint64(_C1_INV)
        z = _unxorshift(z, 30)
    return z


def keys_for_fingerprints(fps: np.ndarray, q: int, r: int, seed: int = 7) -> np.ndarray:
    """Keys whose p = q + r low hash bits equal fps (random high bits)."""
    fps = np.asarray(fps, dtype=np.uint64)
    p = q + r
    g = np.random.Generator(np.random.PCG64(seed))
    hi = g.integers(0, 1 << (64 - p), size=len(fps), dtype=np.uint64) if p < 64 else np.zeros(len(fps), np.uint64)
    h = (hi << np.uint64(p)) | fps if p < 64 else fps
    return fin64_inverse(h)
