"""Mixed-shape workloads: every codeword draws its base graph, lift and
number of kept rows, and the batch is grouped by shape.

Codeword i of seed d draws (bg, Z, rows) from the keyed stream (d, 11, i):
bg uniform in {1, 2}, Z uniform in LIFTS, rows uniform in [4, M_bg]; its
data (information bits, noise) come from the channel stream (d, i) at the
given Eb/N0 with sigma^2 from its own rate. Inputs only: no decoding
arithmetic here.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .channel import Batch, make_batch
from .graph import LIFTS, full_shape, make_graph
from .prng import stream


@dataclasses.dataclass
class ShapeGroup:
    bg: int
    Z: int
    rows: int
    indices: np.ndarray  # global codeword indices in this group
    batch: Batch


def draw_shapes(n_cw: int, seed: int, lifts=LIFTS):
    out = np.empty((n_cw, 3), dtype=np.int64)
    for i in range(n_cw):
        s = stream(seed, 11, i)
        bg = int(s.integers(1, 3))
        Z = int(lifts[int(s.integers(0, len(lifts)))])
        rows = int(s.integers(4, full_shape(bg)[0] + 1))
        out[i] = (bg, Z, rows)
    return out


def make_mixed(n_cw: int, ebn0_db, seed: int, lifts=LIFTS) -> list[ShapeGroup]:
    """Codewords 0..n_cw-1 of seed ``seed`` grouped by (bg, Z, rows)."""
    shapes = draw_shapes(n_cw, seed, lifts)
    groups = []
    keys = sorted({tuple(x) for x in shapes.tolist()})
    for bg, Z, rows in keys:
        idx = np.nonzero((shapes[:, 0] == bg) & (shapes[:, 1] == Z) & (shapes[:, 2] == rows))[0]
        g = make_graph(bg, Z, rows)
        groups.append(ShapeGroup(bg, Z, rows, idx, make_batch(g, len(idx), ebn0_db, seed,
                                                              indices=idx)))
    return groups
