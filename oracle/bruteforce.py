"""Exhaustive-search references for tiny codes -- TEST INFRASTRUCTURE ONLY.

For a code small enough to list every codeword, these give the maximum-
likelihood codeword, the max-log-MAP and the exact MAP bit LLRs by
definition (no message passing), so they check the oracle from outside: on a
cycle-free Tanner graph min-sum with beta = 1 is exact max-log-MAP (paper
§III's min-sum approximation becomes exact when the graph is a tree) and
sum-product belief propagation is exact MAP.
"""
from __future__ import annotations

import itertools

import numpy as np


def gf2_nullspace(H: np.ndarray) -> np.ndarray:
    """Basis (rows) of {c : H c = 0 over GF(2)}."""
    H = (np.asarray(H, dtype=np.uint8) & 1).copy()
    m, n = H.shape
    pivots = []
    row = 0
    for col in range(n):
        if row >= m:
            break
        nz = np.nonzero(H[row:, col])[0]
        if nz.size == 0:
            continue
        p = row + nz[0]
        H[[row, p]] = H[[p, row]]
        for r in range(m):
            if r != row and H[r, col]:
                H[r] ^= H[row]
        pivots.append(col)
        row += 1
    free = [c for c in range(n) if c not in pivots]
    basis = []
    for f in free:
        v = np.zeros(n, dtype=np.uint8)
        v[f] = 1
        for i, pc in enumerate(pivots):
            v[pc] = H[i, f]
        basis.append(v)
    return np.array(basis, dtype=np.uint8).reshape(len(basis), n)


def all_codewords(H: np.ndarray) -> np.ndarray:
    """Every codeword of the code with parity-check matrix H (small only)."""
    B = gf2_nullspace(H)
    k = B.shape[0]
    if k > 20:
        raise ValueError("code too large for exhaustive listing")
    words = []
    for coeffs in itertools.product((0, 1), repeat=k):
        c = np.zeros(H.shape[1], dtype=np.uint8)
        for a, b in zip(coeffs, B):
            if a:
                c ^= b
        words.append(c)
    return np.array(words, dtype=np.uint8)


def correlation(words: np.ndarray, llr: np.ndarray) -> np.ndarray:
    """Sum_i (1 - 2 c_i) L_i / 2 for every codeword (the log-likelihood up to
    a constant, with L = log P(0)/P(1))."""
    return ((1.0 - 2.0 * words.astype(np.float64)) @ np.asarray(llr, np.float64)) / 2.0


def ml_codeword(words: np.ndarray, llr: np.ndarray) -> np.ndarray:
    return words[int(np.argmax(correlation(words, llr)))]


def maxlog_map(words: np.ndarray, llr: np.ndarray) -> np.ndarray:
    """Max-log-MAP LLR of each bit:
    max_{c: c_j = 0} corr(c) - max_{c: c_j = 1} corr(c)."""
    corr = correlation(words, llr)
    out = np.empty(words.shape[1])
    for j in range(words.shape[1]):
        out[j] = corr[words[:, j] == 0].max() - corr[words[:, j] == 1].max()
    return out


def exact_map(words: np.ndarray, llr: np.ndarray) -> np.ndarray:
    """Exact bitwise MAP LLR of each bit, log P(c_j = 0 | y) / P(c_j = 1 | y)
    = logsumexp_{c: c_j = 0} corr(c) - logsumexp_{c: c_j = 1} corr(c) (what
    sum-product belief propagation computes exactly on a cycle-free graph)."""
    corr = correlation(words, llr)
    out = np.empty(words.shape[1])
    for j in range(words.shape[1]):
        a, b = corr[words[:, j] == 0], corr[words[:, j] == 1]
        out[j] = (a.max() + np.log(np.exp(a - a.max()).sum())) - \
                 (b.max() + np.log(np.exp(b - b.max()).sum()))
    return out
