"""Input generators: graph shape invariants, encoders, channel statistics."""
import numpy as np
import pytest

from synth import (ElimEncoder, encode, full_shape, make_batch, make_graph, sigma2, syndrome)
from synth.encoder import _gf2_solve_matrix


@pytest.mark.parametrize("bg", [1, 2])
def test_graph_shape(bg):
    m, n, kb = full_shape(bg)
    g = make_graph(bg, 384)
    assert (g.M, g.N, g.kb) == (m, n, kb)
    w = g.row_weights()
    if bg == 1:
        # 121 kB of int8 messages at Z = 384 (paper §IV) is 316 blocks.
        assert g.E == 316 and g.E * 384 == 121344
        # row weights span 3..19 (paper §IV)
        assert w.min() == 3 and w.max() == 19
    else:
        assert g.E == 197 and w.max() <= 10
    for r, c, s in g.edges():
        assert 0 <= s < g.Z
    base = g.dense_base()
    # punctured columns: column 0 in every core row, column 1 not in core row 1
    assert all(base[r, 0] >= 0 for r in range(4))
    assert base[1, 1] < 0 and all(base[r, 1] >= 0 for r in (0, 2, 3))
    # dual-diagonal core and identity extension
    assert base[0, kb] == base[3, kb] and base[1, kb] == 0
    for r in range(4, m):
        assert base[r, kb + r] == 0
        assert (base[r, kb + 4:] >= 0).sum() == 1
    # column degrees: extension parity columns have degree one
    deg = (base >= 0).sum(axis=0)
    assert (deg[kb + 4:] == 1).all()


def test_graph_deterministic_and_nested():
    a = make_graph(1, 96)
    b = make_graph(1, 96)
    assert a.digest() == b.digest()
    assert make_graph(1, 96, seed=1).digest() != a.digest()
    s = a.sub(10)
    assert s.M == 10 and s.N == 32 and s.E == int(a.row_ptr[10])
    assert (s.col < s.N).all()


@pytest.mark.parametrize("bg,Z", [(2, 16), (1, 16), (2, 32)])
def test_structured_encoder_matches_elimination(bg, Z):
    rng = np.random.default_rng(0)
    g = make_graph(bg, Z)
    u = rng.integers(0, 2, (8, g.K), dtype=np.uint8)
    H = g.dense_H().astype(np.int64)
    for M in (4, 5, 11, g.M):
        gs = g.sub(M)
        c = encode(gs, u)
        assert (c[:, :g.K] == u).all()
        Hs = gs.dense_H().astype(np.int64)
        assert not ((Hs @ c.T.astype(np.int64)) % 2).any()
        ce = ElimEncoder(gs).encode(u)
        assert (ce == c).all()
    # nesting: the M-row codeword is a prefix of the full one
    cf = encode(g, u)
    c6 = encode(g.sub(6), u)
    assert (cf[:, :c6.shape[1]] == c6).all()
    assert not ((H @ cf.T.astype(np.int64)) % 2).any()


def test_encoder_linear_and_syndrome():
    g = make_graph(1, 64)
    rng = np.random.default_rng(1)
    u1 = rng.integers(0, 2, (3, g.K), dtype=np.uint8)
    u2 = rng.integers(0, 2, (3, g.K), dtype=np.uint8)
    assert ((encode(g, u1) ^ encode(g, u2)) == encode(g, u1 ^ u2)).all()
    assert not syndrome(g, encode(g, u1)).any()
    c = encode(g, u1)
    c[0, 5] ^= 1
    assert syndrome(g, c)[0].any()


def test_gf2_solve():
    rng = np.random.default_rng(3)
    while True:
        A = rng.integers(0, 2, (12, 12), dtype=np.uint8)
        try:
            X = _gf2_solve_matrix(A, np.eye(12, dtype=np.uint8))
            break
        except ValueError:
            continue
    assert ((A.astype(int) @ X.astype(int)) % 2 == np.eye(12)).all()


def test_channel_statistics_small_config():
    # BG2-shaped Z=16 at Eb/N0 = 2 dB: q*(1-2c) has mean 8/sigma^2 and
    # standard deviation 8/sigma before rounding and clipping.
    g = make_graph(2, 16)
    b = make_batch(g, 1000, 2.0, data_seed=1)
    s2 = sigma2(g.rate, 2.0)
    assert abs(s2 - 1.5774) < 1e-3
    tx = b.c[:, 2 * g.Z:].astype(np.float64)
    v = b.q.astype(np.float64) * (1 - 2 * tx)
    assert abs(v.mean() - 8 / s2) < 0.05
    assert abs(v.std() - 8 / np.sqrt(s2)) < 0.05
    assert b.q.min() >= -127 and b.q.max() <= 127
    assert not syndrome(g, b.c).any()


def test_channel_reproducible_under_split():
    g = make_graph(2, 32)
    full = make_batch(g, 10, 1.5, data_seed=9)
    part = make_batch(g, 4, 1.5, data_seed=9, start=3)
    assert (full.q[3:7] == part.q).all() and (full.u[3:7] == part.u).all()
