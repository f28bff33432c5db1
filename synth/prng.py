"""Keyed counter-based random streams for the synthetic workloads.

Every random draw in the workloads (graph shifts, information bits, channel
noise) comes from a Philox4x64-10 stream (Salmon et al., "Parallel random
numbers: as easy as 1, 2, 3", SC'11) whose 128-bit key is built from a seed
and the identity of the object being drawn (a codeword index, a base graph).
A codeword's data therefore depends only on (seed, index), never on batch
size, batch split or thread count.

This module holds no decoding arithmetic; it is shared by the CPU oracle's
tests and by the GPU path's tests and benchmark as a source of inputs only.
"""
from __future__ import annotations

import numpy as np

_MASK64 = (1 << 64) - 1


def stream(seed: int, *ids: int) -> np.random.Generator:
    """Return an independent generator keyed by ``seed`` and up to one 64-bit
    id word built from ``ids`` (each id < 2**16 except the last, which may use
    the remaining bits)."""
    word = 0
    for i in ids[:-1]:
        if not 0 <= i < (1 << 16):
            raise ValueError("ids other than the last must be < 2**16")
        word = (word << 16) | int(i)
    if ids:
        last = int(ids[-1])
        if last < 0:
            raise ValueError("ids must be non-negative")
        word = ((word << 40) | last) & _MASK64
    key = np.array([int(seed) & _MASK64, word], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))
