"""GF(2) encoders for the synthetic quasi-cyclic codes.

Two independent encoders produce the systematic codeword c = [u | p]
(u = K_b·Z information bits, p = M·Z parity bits) with H·c = 0:

* ``ElimEncoder`` -- Gaussian elimination of the lifted H over GF(2): it
  solves H_p·p = H_u·u once for a generator of the parity part. It works for
  any full-rank parity part and is meant for small lifts (the BG2-shaped Z=16
  workload) and as the check of the structured encoder.
* ``encode`` -- the structured encoder that follows the dual-diagonal core
  and the identity-extended lower part of the generated graphs, in O(E·Z)
  per codeword, vectorised over a batch.

Variables are ordered column-block-major: bit j = c·Z + z.
Circulant convention: block (r, c, s) maps row z to variable (z + s) mod Z.
This module is an input generator: it holds none of the decoding arithmetic.
"""
from __future__ import annotations

import numpy as np

from .graph import BaseGraph


def _shifted(v: np.ndarray, s: int) -> np.ndarray:
    """(P^s v)[..., z] = v[..., (z + s) mod Z] along the last axis."""
    return np.roll(v, -s, axis=-1) if s else v


def encode(g: BaseGraph, u: np.ndarray) -> np.ndarray:
    """Structured encoder: u uint8 [B, K_b*Z] (0/1) -> c uint8 [B, N*Z]."""
    if g.n_punct != 2:
        raise ValueError("structured encoder needs a BG-shaped graph")
    u = np.asarray(u, dtype=np.uint8)
    B = u.shape[0]
    Z, kb, M = g.Z, g.kb, g.M
    if M < 4:
        raise ValueError("structured encoder needs the four core rows")
    x = np.zeros((B, g.N, Z), dtype=np.uint8)
    x[:, :kb, :] = u.reshape(B, kb, Z)
    lam = np.zeros((4, B, Z), dtype=np.uint8)
    a = None
    for r, c, s in g.edges():
        if r >= 4:
            break
        if c < kb:
            lam[r] ^= _shifted(x[:, c, :], s)
        elif c == kb and r == 0:
            a = s
    assert a is not None
    p0 = lam[0] ^ lam[1] ^ lam[2] ^ lam[3]
    p1 = lam[0] ^ _shifted(p0, a)
    p2 = lam[1] ^ p0 ^ p1
    p3 = lam[3] ^ _shifted(p0, a)
    x[:, kb] = p0
    x[:, kb + 1] = p1
    x[:, kb + 2] = p2
    x[:, kb + 3] = p3
    for r in range(4, M):
        acc = np.zeros((B, Z), dtype=np.uint8)
        ident = kb + r
        for e in range(g.row_ptr[r], g.row_ptr[r + 1]):
            c, s = int(g.col[e]), int(g.shift[e])
            if c == ident:
                if s != 0:
                    raise ValueError("extension block must be an identity")
                continue
            acc ^= _shifted(x[:, c, :], s)
        x[:, ident] = acc
    return x.reshape(B, g.N * Z)


def _gf2_solve_matrix(A: np.ndarray, Bm: np.ndarray) -> np.ndarray:
    """Return X with A·X = Bm over GF(2) (A square, full rank)."""
    n = A.shape[0]
    W = np.concatenate([A, Bm], axis=1).astype(np.uint8)
    for col in range(n):
        piv = col + int(np.argmax(W[col:, col]))
        if W[piv, col] == 0:
            raise ValueError("parity part of H is singular")
        if piv != col:
            W[[col, piv]] = W[[piv, col]]
        rows = np.nonzero(W[:, col])[0]
        rows = rows[rows != col]
        if rows.size:
            W[rows] ^= W[col]
    return W[:, n:]


class ElimEncoder:
    """Encoder by Gaussian elimination of the lifted parity-check matrix."""

    def __init__(self, g: BaseGraph):
        H = g.dense_H()
        K = g.K
        self.g = g
        Hu, Hp = H[:, :K], H[:, K:]
        if Hp.shape[0] != Hp.shape[1]:
            raise ValueError("H must have as many check rows as parity bits")
        # p = Hp^{-1} Hu u  (GF(2)); store the dense parity generator.
        self.P = _gf2_solve_matrix(Hp, Hu)  # [M*Z, K]

    def encode(self, u: np.ndarray) -> np.ndarray:
        u = np.asarray(u, dtype=np.uint8)
        p = (u.astype(np.int64) @ self.P.T.astype(np.int64)) & 1
        return np.concatenate([u, p.astype(np.uint8)], axis=1)


def syndrome(g: BaseGraph, c: np.ndarray) -> np.ndarray:
    """H·c over GF(2) for c uint8 [B, N*Z] -> uint8 [B, M*Z]."""
    c = np.asarray(c, dtype=np.uint8)
    B = c.shape[0]
    x = c.reshape(B, g.N, g.Z)
    s = np.zeros((B, g.M, g.Z), dtype=np.uint8)
    for r, col, sh in g.edges():
        s[:, r] ^= _shifted(x[:, col, :], sh)
    return s.reshape(B, g.M * g.Z)
