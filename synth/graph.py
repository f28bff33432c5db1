"""Seeded BG1/BG2-shaped quasi-cyclic base graphs.

The 5G NR codes are quasi-cyclic: a base matrix of M_bg x (K_b + M_bg) blocks,
each either zero or a Z x Z cyclic-shift permutation, lifted by Z (paper
§II). The standard's shift tables are not reproduced here; these graphs have
the same shapes (BG1 46 x 68 with K_b = 22 and 316 nonzero blocks, the number
implied by the 121 kB int8 message store of §IV at Z = 384; BG2 42 x 52 with
K_b = 10), the same dual-diagonal parity core and the same identity-extended
lower part, with every free shift drawn uniformly in [0, Z) from a keyed
counter-based stream.

Circulant convention: block (r, c) with shift s connects check row z of
block row r to variable (z + s) mod Z of block column c.

Structure of the full graph (rows r, columns c):

* core rows 0..3 -- random information columns plus the parity core
  p0 = column K_b in rows {0, 1, 3} with shifts (a, 0, a), p1 = K_b + 1 in
  rows {0, 1}, p2 = K_b + 2 in rows {1, 2}, p3 = K_b + 3 in rows {2, 3}
  (shift 0). Summing the four block rows leaves p0 alone, so the core is
  invertible for every Z and every a.
* column 0 (punctured) is in every core row, column 1 (punctured) in core
  rows 0, 2 and 3 only, so both punctured columns are recovered in the first
  iteration of a layered decoder even when only the four core rows are kept.
* extension row r >= 4 -- an identity block at column K_b + r plus a few
  random columns in [0, K_b + 4); row 4 holds column 0 but not 1, row 5
  column 1 but not 0.

Keeping the first M rows (4 <= M <= M_bg) and the first K_b + M columns gives
the nested rate-K_b/(K_b + M - 2) sub-codes.

This module is an input generator: it holds none of the decoding arithmetic.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

from .prng import stream

GRAPH_SEED = 200905534
LIFTS = (16, 32, 64, 96, 128, 192, 256, 384)

# (rows, cols, K_b, core info-column counts per core row, total nonzero blocks)
_SHAPES = {
    1: (46, 68, 22, (17, 16, 17, 17), 316),
    2: (42, 52, 10, (6, 7, 6, 6), 197),
}
_TAG_STRUCTURE = 1
_TAG_SHIFTS = 2


def full_shape(bg: int) -> tuple[int, int, int]:
    """(M_bg, N_bg, K_b) of the full base graph ``bg``."""
    m, n, kb, _, _ = _SHAPES[bg]
    return m, n, kb


@dataclasses.dataclass(frozen=True)
class BaseGraph:
    """A lifted base graph restricted to its first ``M`` rows.

    ``row_ptr[r]:row_ptr[r + 1]`` indexes the blocks of row r in ascending
    column order; ``col`` and ``shift`` give each block's column and shift.
    """

    bg: int
    Z: int
    M: int
    N: int
    kb: int
    row_ptr: np.ndarray  # int32 [M + 1]
    col: np.ndarray  # int16 [E]
    shift: np.ndarray  # int16 [E]
    n_punct: int = 2

    @property
    def E(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def K(self) -> int:
        return self.kb * self.Z

    @property
    def Nc(self) -> int:
        return self.N * self.Z

    @property
    def T(self) -> int:
        """Number of transmitted (non-punctured) code bits."""
        return (self.N - self.n_punct) * self.Z

    @property
    def rate(self) -> float:
        return self.kb / (self.N - self.n_punct)

    def row_weights(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edges(self):
        """Yield (row, col, shift) for every nonzero block, row-major."""
        for r in range(self.M):
            for e in range(self.row_ptr[r], self.row_ptr[r + 1]):
                yield r, int(self.col[e]), int(self.shift[e])

    def sub(self, M: int) -> "BaseGraph":
        """The nested sub-code keeping the first ``M`` block rows."""
        if not 1 <= M <= self.M:
            raise ValueError(f"M={M} out of range 1..{self.M}")
        e = int(self.row_ptr[M])
        return dataclasses.replace(
            self, M=M, N=self.kb + M if self.n_punct == 2 else self.N,
            row_ptr=self.row_ptr[: M + 1].copy(), col=self.col[:e].copy(),
            shift=self.shift[:e].copy())

    def dense_base(self) -> np.ndarray:
        """Base matrix with -1 for zero blocks and the shift otherwise."""
        b = -np.ones((self.M, self.N), dtype=np.int32)
        for r, c, s in self.edges():
            b[r, c] = s
        return b

    def dense_H(self) -> np.ndarray:
        """The lifted parity-check matrix as a uint8 0/1 array (small Z only)."""
        H = np.zeros((self.M * self.Z, self.N * self.Z), dtype=np.uint8)
        z = np.arange(self.Z)
        for r, c, s in self.edges():
            H[r * self.Z + z, c * self.Z + (z + s) % self.Z] = 1
        return H

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (np.array([self.bg, self.Z, self.M, self.N, self.kb, self.n_punct], np.int64),
                  self.row_ptr.astype(np.int64), self.col.astype(np.int64),
                  self.shift.astype(np.int64)):
            h.update(a.tobytes())
        return h.hexdigest()[:16]


def _structure(bg: int, seed: int):
    """Row -> sorted list of (column, kind) for the full base graph; kind is
    'free' for a block whose shift is drawn, or a fixed shift code."""
    m, n, kb, core_info, total = _SHAPES[bg]
    g = stream(seed, _TAG_STRUCTURE, bg)
    rows: list[dict[int, str]] = []
    # Core rows: information columns.
    while True:
        core = []
        for r in range(4):
            forced = {0} | ({1} if r != 1 else set())
            banned = {1} if r == 1 else set()
            pool = [c for c in range(kb) if c not in forced and c not in banned]
            extra = g.choice(pool, size=core_info[r] - len(forced), replace=False)
            core.append(forced | {int(c) for c in extra})
        if set().union(*core) == set(range(kb)):
            break
    for r in range(4):
        rows.append({c: "free" for c in core[r]})
    # Parity core.
    rows[0][kb] = "a"
    rows[1][kb] = "zero"
    rows[3][kb] = "a"
    rows[0][kb + 1] = "zero"
    rows[1][kb + 1] = "zero"
    rows[1][kb + 2] = "zero"
    rows[2][kb + 2] = "zero"
    rows[2][kb + 3] = "zero"
    rows[3][kb + 3] = "zero"
    core_edges = sum(len(x) for x in rows)
    # Extension rows: number of random columns per row, summing to the total.
    n_ext = m - 4
    extra_total = total - core_edges - n_ext
    lo, hi = 2, 9
    # Heavier rows first, tapering towards the low-rate end (as in the
    # standard's lower part), scaled to the edge total.
    profile = np.linspace(hi - 1, lo, n_ext)
    d = np.clip(np.round(profile * extra_total / profile.sum()), lo, hi).astype(np.int64)
    rem = extra_total - int(d.sum())
    while rem != 0:
        i = int(g.integers(0, n_ext))
        step = 1 if rem > 0 else -1
        if lo <= d[i] + step <= hi:
            d[i] += step
            rem -= step
    assert lo <= d.min() and d.max() <= hi and int(d.sum()) == extra_total
    width = kb + 4
    for i in range(n_ext):
        r = 4 + i
        row = {kb + r: "zero"}
        if r == 4:
            forced, banned = {0}, {1}
        elif r == 5:
            forced, banned = {1}, {0}
        else:
            forced, banned = set(), set()
        pool = [c for c in range(width) if c not in forced and c not in banned]
        extra = g.choice(pool, size=int(d[i]) - len(forced), replace=False)
        for c in forced | {int(c) for c in extra}:
            row[c] = "free"
        rows.append(row)
    assert sum(len(x) for x in rows) == total
    return rows


def make_graph(bg: int, Z: int, M: int | None = None, seed: int = GRAPH_SEED) -> BaseGraph:
    """The seeded BG-shaped base graph ``bg`` lifted by ``Z``, first ``M`` rows."""
    if bg not in _SHAPES:
        raise ValueError("bg must be 1 or 2")
    if Z < 1:
        raise ValueError("Z must be >= 1")
    m, n, kb, _, _ = _SHAPES[bg]
    rows = _structure(bg, seed)
    gs = stream(seed, _TAG_SHIFTS, bg, Z)
    a = int(gs.integers(0, Z))
    row_ptr = [0]
    cols: list[int] = []
    shifts: list[int] = []
    for r in range(m):
        for c in sorted(rows[r]):
            kind = rows[r][c]
            s = int(gs.integers(0, Z))  # always drawn so the stream stays aligned
            if kind == "zero":
                s = 0
            elif kind == "a":
                s = a
            cols.append(c)
            shifts.append(s)
        row_ptr.append(len(cols))
    full = BaseGraph(bg=bg, Z=Z, M=m, N=n, kb=kb,
                     row_ptr=np.array(row_ptr, np.int32),
                     col=np.array(cols, np.int16), shift=np.array(shifts, np.int16))
    return full if M is None or M == m else full.sub(M)


def make_toy_graph(base: np.ndarray, Z: int, kb: int, n_punct: int = 0) -> BaseGraph:
    """A graph from an explicit base matrix (-1 = zero block), for small tests."""
    base = np.asarray(base)
    M, N = base.shape
    row_ptr = [0]
    cols, shifts = [], []
    for r in range(M):
        for c in range(N):
            if base[r, c] >= 0:
                cols.append(c)
                shifts.append(int(base[r, c]) % Z)
        row_ptr.append(len(cols))
    return BaseGraph(bg=0, Z=Z, M=M, N=N, kb=kb, row_ptr=np.array(row_ptr, np.int32),
                     col=np.array(cols, np.int16), shift=np.array(shifts, np.int16),
                     n_punct=n_punct)
