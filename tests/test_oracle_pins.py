"""Pins of the CPU oracle against facts fixed outside it: hand-computed
messages, exhaustive max-log-MAP / ML search on tiny codes, the encoder
(valid codewords), IEEE binary16 rounding as implemented by numpy, and exact
invariants of the algorithm. None of these retypes the oracle's formulas."""
import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from synth import (encode, make_batch, make_graph, make_toy_graph, noiseless_q, quantize,
                   syndrome)
from synth.channel import sigma2


def one_row(Z=1, w=4, shifts=None):
    base = np.array([shifts if shifts is not None else [0] * w])
    return make_toy_graph(base, Z=Z, kb=w - 1, n_punct=0)


# --------------------------------------------------------------------------
# Hand-computed single-row update (min-sum with beta = 3/4 in Q1.7,
# round half up, symmetric saturation at +-127).
# --------------------------------------------------------------------------

def _row_llr(q, iters, **kw):
    g = one_row()
    _, _, _, llr = oracle.decode_i8(g, np.array([q], np.int8), max_iter=iters, early_exit=False,
                                    want_llr=True, **kw)
    return llr[0].tolist()


def test_hand_example_one_row():
    # L = [10, -3, 7, -20], R = 0: m1 = 3 (edge 1), m2 = 7, sign product +;
    # a1 = (3*3 + 2) >> 2 = 2, a2 = (3*7 + 2) >> 2 = 5 -> R' = [2, -5, 2, -2].
    assert _row_llr([10, -3, 7, -20], 1) == [12, -8, 9, -22]
    # Re-running the same row changes nothing when nothing saturated.
    assert _row_llr([10, -3, 7, -20], 2) == [12, -8, 9, -22]


def test_hand_example_offset():
    # offset 2 before normalisation: m1 -> 1, m2 -> 5; a1 = 1, a2 = 4.
    assert _row_llr([10, -3, 7, -20], 1, delta=2) == [11, -7, 8, -21]


def test_hand_example_saturation_order():
    # Iteration 1: m1 = 120, m2 = 124, a1 = 90, a2 = 93 -> L' saturates at 127.
    # Iteration 2 sees x = 127 - R = [37, 34, 37, 37]: m1 = 34, m2 = 37,
    # a1 = 26, a2 = 28 -> [63, 62, 63, 63]. Without the clamp after the add,
    # iteration 2 would repeat iteration 1.
    assert _row_llr([126, 120, 125, 124], 1) == [127, 127, 127, 127]
    assert _row_llr([126, 120, 125, 124], 2) == [63, 62, 63, 63]
    # The clamp is symmetric: -127, never -128.
    assert _row_llr([-126, -120, -125, -124], 1) == [-127, -127, -127, -127]
    assert _row_llr([-126, -120, -125, -124], 2) == [-63, -62, -63, -63]
    # An input of -128 is read as -127: with beta = 1 the only other edge
    # then receives 127 in magnitude.
    g = one_row(w=2)
    _, _, _, llr = oracle.decode_i8(g, np.array([[-128, 0]], np.int8), max_iter=1,
                                    early_exit=False, want_llr=True,
                                    wq=np.full((1, 1), 128, np.uint8))
    assert llr[0].tolist() == [-127, -127]


def test_hand_example_fp16():
    # Same row in binary16: a1 = 0.75*3 = 2.25, a2 = 0.75*7 = 5.25 (exact).
    g = one_row()
    _, _, _, llr = oracle.decode_f16(g, np.array([[10, -3, 7, -20]], np.int8), max_iter=1,
                                     early_exit=False, want_llr=True)
    assert oracle.f16_to_f64(llr[0]).tolist() == [12.25, -8.25, 9.25, -22.25]


def test_hand_example_fp16_rounding():
    # A row where every binary16 operation of the update rounds: the
    # normalisation's offset subtraction and product, the extrinsic
    # subtraction L - R and the posterior sum x + R' (rounding to nearest,
    # ties to even). One check on three bits, L = [42, -13, -87],
    # w = rn16(2.9) = 2.900390625 (0x41CD), offset rn16(0.3) =
    # 0.300048828125 (0x34CD), two iterations, no early exit.
    #
    # Iteration 1 (R = 0, x = L): |x| = [42, 13, 87], m1 = 13 (edge 1),
    # m2 = 42, sign product + (two negatives).
    #   m1 - off = 12.699951171875 -> 12.703125 (quantum 2^-7);
    #   w * 12.703125 = 36.844024658203125 -> a1 = 36.84375 (2^-5)
    #   m2 - off = 41.699951171875 -> 41.6875 (2^-5);
    #   w * 41.6875 = 120.9100341796875 -> a2 = 120.9375 (2^-4)
    #   R' = [+a1, -a2, -a1] (edge k gets the sign of x_k times the product)
    #   L' = [42 + 36.84375 = 78.84375 -> 78.875 (2^-4),
    #         -13 - 120.9375 = -133.9375 -> -134.0 (2^-3, a tie: to even),
    #         -87 - 36.84375 = -123.84375 -> -123.875 (2^-4)]
    # Iteration 2: x = L' - R' = [78.875 - 36.84375 = 42.03125 (exact),
    #   -134 + 120.9375 = -13.0625 (exact), -123.875 + 36.84375 = -87.03125
    #   -> -87.0 (2^-4, a tie: to even)]; m1 = 13.0625, m2 = 42.03125
    #   m1 - off = 12.762451171875 -> 12.765625; w * 12.765625 =
    #   37.025299072265625 -> a1 = 37.03125
    #   m2 - off = 41.731201171875 -> 41.71875; w * 41.71875 =
    #   121.00067138671875 -> a2 = 121.0
    #   L' = [42.03125 + 37.03125 = 79.0625 (exact),
    #         -13.0625 - 121 = -134.0625 -> -134.0 (2^-3, a tie: to even),
    #         -87.0 - 37.03125 = -124.03125 -> -124.0 (2^-3)]
    # Keeping any one of the four operations unrounded changes the result
    # (e.g. an unrounded L - R gives -124.0625 for the last bit).
    g = one_row(w=3)
    q = np.array([[42, -13, -87]], np.int8)
    for iters, want in ((1, [78.875, -134.0, -123.875]), (2, [79.0625, -134.0, -124.0])):
        _, _, _, llr = oracle.decode_f16(g, q, max_iter=iters, early_exit=False, beta=2.9,
                                         delta=0.3, want_llr=True)
        assert oracle.f16_to_f64(llr[0]).tolist() == want
    # the same steps in numpy's IEEE binary16 arithmetic, one operation at a time
    h = np.float16
    w, off = h(2.9), h(0.3)
    a1, a2 = w * (h(13) - off), w * (h(42) - off)
    L1 = [h(42) + a1, h(-13) - a2, h(-87) - a1]
    x = [L1[0] - a1, L1[1] + a2, L1[2] + a1]
    b1, b2 = w * (abs(x[1]) - off), w * (abs(x[0]) - off)
    L2 = [x[0] + b1, x[1] - b2, x[2] - b1]
    assert [float(v) for v in L1] == [78.875, -134.0, -123.875]
    assert [float(v) for v in L2] == [79.0625, -134.0, -124.0]
    # per-(iteration, row) weights take the same path as a scalar beta
    wh = np.full((2, 1), 0x41CD, np.uint16)
    _, _, _, llr = oracle.decode_f16(g, q, max_iter=2, early_exit=False, wh=wh, delta=0.3,
                                     want_llr=True)
    assert oracle.f16_to_f64(llr[0]).tolist() == [79.0625, -134.0, -124.0]


# --------------------------------------------------------------------------
# binary16 rounding against numpy's IEEE conversion
# --------------------------------------------------------------------------

def test_f16_rounding_matches_numpy():
    rng = np.random.default_rng(0)
    v = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 5, 20000),
        np.arange(-3000, 3000) * 0.125 + 0.0625,           # ties at several scales
        np.array([65504.0, 65519.99, 65520.0, 1e6, -1e6, 2.0 ** -24, 2.0 ** -25,
                  3 * 2.0 ** -26, 2.0 ** -14 - 2.0 ** -25, 0.0, -0.0]),
    ])
    ref = v.astype(np.float16).view(np.uint16)
    assert (oracle.f64_to_f16(v) == ref).all()
    h = np.arange(65536, dtype=np.uint16)
    finite = (h & 0x7C00) != 0x7C00
    back = oracle.f16_to_f64(h[finite])
    assert (back == h[finite].view(np.float16).astype(np.float64)).all()
    assert (oracle.f64_to_f16(back) == h[finite]).all()


# --------------------------------------------------------------------------
# Single parity check and trees against exhaustive max-log-MAP
# --------------------------------------------------------------------------

@pytest.mark.parametrize("w", [2, 3, 5, 8])
def test_spc_is_maxlog_map(w):
    # One check is a tree: one layer of min-sum with beta = 1 gives the exact
    # max-log-MAP posterior of every bit.
    rng = np.random.default_rng(w)
    g = one_row(w=w)
    words = bf.all_codewords(g.dense_H())
    for _ in range(20):
        q = rng.integers(-60, 61, (1, w)).astype(np.int8)
        _, _, _, llr = oracle.decode_i8(g, q, max_iter=1, early_exit=False, want_llr=True,
                                        wq=np.full((1, 1), 128, np.uint8))
        assert llr[0].tolist() == bf.maxlog_map(words, q[0].astype(float)).tolist()
        lf = rng.standard_normal((1, w)) * 3
        _, _, _, l64 = oracle.decode_f64(g, lf, max_iter=1, early_exit=False, beta=1.0,
                                         want_llr=True)
        assert np.allclose(l64[0], bf.maxlog_map(words, lf[0]), rtol=0, atol=1e-12)


TREE = np.array([
    # a cycle-free base graph: 4 checks, 9 variables, 12 edges, connected
    [0, 0, 0, -1, -1, -1, -1, -1, -1],
    [-1, -1, 0, 0, 0, -1, -1, -1, -1],
    [-1, -1, -1, -1, 0, 0, 0, -1, -1],
    [-1, 0, -1, -1, -1, -1, -1, 0, 0],
])


@pytest.mark.parametrize("Z", [1, 3])
def test_tree_is_maxlog_map(Z):
    rng = np.random.default_rng(10 + Z)
    base = np.where(TREE >= 0, rng.integers(0, Z, TREE.shape), -1)
    g = make_toy_graph(base, Z=Z, kb=5)  # a lift of a tree is a forest
    words = bf.all_codewords(g.dense_H())
    for _ in range(10):
        lf = rng.standard_normal((1, g.N * Z)) * 2
        _, _, _, l64 = oracle.decode_f64(g, lf, max_iter=12, early_exit=False, beta=1.0,
                                         want_llr=True)
        assert np.allclose(l64[0], bf.maxlog_map(words, lf[0]), atol=1e-9)
        qi = rng.integers(-20, 21, (1, g.N * Z)).astype(np.int8)
        _, _, _, li = oracle.decode_i8(g, qi, max_iter=12, early_exit=False, want_llr=True,
                                       wq=np.full((1, g.M), 128, np.uint8))
        assert li[0].tolist() == bf.maxlog_map(words, qi[0].astype(float)).tolist()
        _, _, _, lh = oracle.decode_f16(g, qi, max_iter=12, early_exit=False, beta=1.0,
                                        want_llr=True)
        assert oracle.f16_to_f64(lh[0]).tolist() == bf.maxlog_map(words, qi[0].astype(float)).tolist()


# --------------------------------------------------------------------------
# BG-shaped codes: noiseless input, symmetry, batch independence
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bg,Z,M", [(2, 16, 42), (2, 16, 4), (1, 16, 46), (1, 32, 7), (2, 64, 20)])
def test_noiseless_decodes_in_one_iteration(bg, Z, M):
    g = make_graph(bg, Z, M)
    u = np.random.default_rng(Z + M).integers(0, 2, (6, g.K), dtype=np.uint8)
    c = encode(g, u)
    q = noiseless_q(c, g)
    for dec in (oracle.decode_i8, oracle.decode_f16):
        bits, iters, ok, _ = dec(g, q, max_iter=10)
        assert (iters == 1).all() and ok.all()
        assert (oracle.unpack_bits(bits, g.K) == u).all()


@pytest.mark.parametrize("bg,Z", [(2, 16), (1, 32)])
def test_codeword_symmetry(bg, Z):
    # Flipping the LLR signs of a valid codeword flips every posterior's sign
    # and nothing else (early exit off), in both number modes.
    g = make_graph(bg, Z)
    rng = np.random.default_rng(5)
    b0 = make_batch(g, 4, 1.0, data_seed=3)
    u = rng.integers(0, 2, (4, g.K), dtype=np.uint8)
    c = encode(g, u)
    # LLRs for the all-zero word: |q| with the noise pattern of b0
    q0 = (b0.q.astype(np.int16) * (1 - 2 * b0.c[:, 2 * Z:].astype(np.int16))).clip(-127, 127)
    sgn = (1 - 2 * c.astype(np.int16))
    qc = (q0 * sgn[:, 2 * Z:]).astype(np.int8)
    _, _, _, l0 = oracle.decode_i8(g, q0.astype(np.int8), max_iter=6, early_exit=False,
                                   want_llr=True)
    _, _, _, lc = oracle.decode_i8(g, qc, max_iter=6, early_exit=False, want_llr=True)
    assert (lc.astype(np.int16) == l0.astype(np.int16) * sgn).all()
    _, _, _, h0 = oracle.decode_f16(g, q0.astype(np.int8), max_iter=6, early_exit=False,
                                    want_llr=True)
    _, _, _, hc = oracle.decode_f16(g, qc, max_iter=6, early_exit=False, want_llr=True)
    assert (oracle.f16_to_f64(hc) == oracle.f16_to_f64(h0) * sgn).all()


def test_batch_order_and_threads_independent():
    g = make_graph(2, 16)
    b = make_batch(g, 40, 1.0, data_seed=1)
    ref = oracle.decode_i8(g, b.q, want_llr=True)
    perm = np.random.default_rng(0).permutation(40)
    got = oracle.decode_i8(g, b.q[perm], want_llr=True, n_threads=4)
    for a, r in zip(got, ref):
        assert (a == r[perm]).all()


def test_plain_equals_q17_weight_96():
    g = make_graph(2, 32)
    b = make_batch(g, 30, 1.0, data_seed=2)
    ref = oracle.decode_i8(g, b.q, want_llr=True)
    got = oracle.decode_i8(g, b.q, want_llr=True, wq=np.full((10, g.M), 96, np.uint8))
    for a, r in zip(got, ref):
        assert (a == r).all()


def test_fp16_equals_f64_when_exact():
    # With beta = 1 and small integer LLRs every binary16 intermediate is an
    # integer below 2048, hence exact: the binary16 mode must then agree
    # with the double mode bit for bit.
    g = make_graph(2, 16, 12)
    rng = np.random.default_rng(7)
    q = rng.integers(-6, 7, (20, g.T)).astype(np.int8)
    _, it64, ok64, l64 = oracle.decode_f64(g, q.astype(np.float64), max_iter=5, beta=1.0,
                                           want_llr=True)
    assert np.abs(l64).max() < 2048 and (l64 == np.round(l64)).all()
    _, it16, ok16, l16 = oracle.decode_f16(g, q, max_iter=5, beta=1.0, want_llr=True)
    assert (oracle.f16_to_f64(l16) == l64).all()
    assert (it16 == it64).all() and (ok16 == ok64).all()


def test_early_exit_and_failure_flags():
    g = make_graph(2, 16)
    b = make_batch(g, 50, -10.0, data_seed=4)  # pure noise: nothing converges
    _, iters, ok, _ = oracle.decode_i8(g, b.q, max_iter=5)
    assert (iters == 5).all() and not ok.any()
    b = make_batch(g, 50, 4.0, data_seed=4)
    bits, iters, ok, llr = oracle.decode_i8(g, b.q, max_iter=10, want_llr=True)
    assert ok.mean() > 0.9
    # ok means the hard decisions satisfy every check
    hd = (llr < 0).astype(np.uint8)
    assert (syndrome(g, hd).any(axis=1) == ~ok).all()
    # without early exit the iteration count is the maximum
    _, iters2, ok2, _ = oracle.decode_i8(g, b.q, max_iter=10, early_exit=False)
    assert (iters2 == 10).all()


# --------------------------------------------------------------------------
# Toy code against brute-force maximum likelihood
# --------------------------------------------------------------------------

def test_toy_code_matches_ml_at_high_snr():
    rng = np.random.default_rng(11)
    Z, kb = 4, 4
    pat = np.array([
        [1, 1, 1, 0, 1, 1, 0, 0],
        [1, 0, 1, 1, 1, 1, 1, 0],
        [1, 1, 0, 1, 0, 0, 1, 1],
        [0, 1, 1, 1, 1, 0, 0, 1],
    ])
    a = int(rng.integers(0, Z))
    base = np.where(pat > 0, rng.integers(0, Z, pat.shape), -1)
    base[:, kb:] = np.where(pat[:, kb:] > 0, 0, -1)
    base[0, kb] = base[3, kb] = a
    g = make_toy_graph(base, Z=Z, kb=kb)
    H = g.dense_H()
    words = bf.all_codewords(H)
    assert words.shape[0] == 2 ** (kb * Z)
    n = 10000
    rate = kb / (g.N)
    s2 = sigma2(rate, 6.0)
    idx = rng.integers(0, words.shape[0], n)
    c = words[idx]
    y = (1 - 2.0 * c) + np.sqrt(s2) * rng.standard_normal(c.shape)
    q = quantize(2 * y / s2)
    _, _, ok, llr = oracle.decode_i8(g, q, max_iter=20, want_llr=True)
    hd = (llr < 0).astype(np.uint8)
    corr = (1.0 - 2.0 * words) @ q.astype(np.float64).T  # [n_words, n]
    ml = words[np.argmax(corr, axis=0)]
    agree = (hd == ml).all(axis=1).mean()
    assert agree >= 0.99
    # whenever the decoder reports success its output is a codeword
    assert not ((H.astype(int) @ hd[ok].T.astype(int)) % 2).any()


# --------------------------------------------------------------------------
# Sum-product rule and flooding schedule (context variants): exact MAP on
# trees, max-log-MAP for min-sum, and the schedules' order properties
# --------------------------------------------------------------------------

@pytest.mark.parametrize("w", [2, 3, 5, 8])
@pytest.mark.parametrize("schedule", ["layered", "flooding"])
def test_spa_single_check_is_exact_map(w, schedule):
    # one check is a tree: one sum-product update gives every bit's exact
    # a-posteriori LLR, whichever schedule
    rng = np.random.default_rng(30 + w)
    g = one_row(w=w)
    words = bf.all_codewords(g.dense_H())
    for _ in range(20):
        lf = rng.standard_normal((1, w)) * 3
        _, _, _, post = oracle.decode_bp(g, lf, rule="spa", schedule=schedule, max_iter=1,
                                         early_exit=False, want_llr=True)
        assert np.allclose(post[0], bf.exact_map(words, lf[0]), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("Z", [1, 3])
@pytest.mark.parametrize("schedule", ["layered", "flooding"])
def test_bp_tree_is_exact(Z, schedule):
    # on a forest, belief propagation run long enough is exact: sum-product
    # gives the MAP LLRs, min-sum with beta = 1 the max-log-MAP LLRs, on
    # either schedule
    rng = np.random.default_rng(40 + Z)
    base = np.where(TREE >= 0, rng.integers(0, Z, TREE.shape), -1)
    g = make_toy_graph(base, Z=Z, kb=5)
    words = bf.all_codewords(g.dense_H())
    for _ in range(10):
        lf = rng.standard_normal((1, g.N * Z)) * 2
        _, _, _, spa = oracle.decode_bp(g, lf, rule="spa", schedule=schedule, max_iter=12,
                                        early_exit=False, want_llr=True)
        assert np.allclose(spa[0], bf.exact_map(words, lf[0]), rtol=1e-10, atol=1e-10)
        _, _, _, ms = oracle.decode_bp(g, lf, rule="minsum", schedule=schedule, beta=1.0,
                                       max_iter=12, early_exit=False, want_llr=True)
        assert np.allclose(ms[0], bf.maxlog_map(words, lf[0]), rtol=0, atol=1e-9)


def test_bp_layered_minsum_equals_double_mode():
    # the min-sum rule on the layered schedule is the decoder's double mode
    g = make_graph(2, 16).sub(12)
    b = make_batch(g, 20, 1.0, data_seed=12)
    lf = b.q.astype(np.float64)
    ref = oracle.decode_f64(g, lf, max_iter=6, beta=0.75, want_llr=True)
    got = oracle.decode_bp(g, lf, rule="minsum", schedule="layered", beta=0.75, max_iter=6,
                           want_llr=True)
    for a, r in zip(got, ref):
        assert np.array_equal(a, r)


def _permute_rows(g, perm):
    rows = [(g.col[g.row_ptr[r]:g.row_ptr[r + 1]], g.shift[g.row_ptr[r]:g.row_ptr[r + 1]])
            for r in perm]
    rp = np.concatenate([[0], np.cumsum([len(c) for c, _ in rows])]).astype(np.int32)
    return type(g)(bg=g.bg, Z=g.Z, M=g.M, N=g.N, kb=g.kb, row_ptr=rp,
                   col=np.concatenate([c for c, _ in rows]).astype(np.int16),
                   shift=np.concatenate([s for _, s in rows]).astype(np.int16))


@pytest.mark.parametrize("rule", ["spa", "minsum"])
def test_flooding_ignores_row_order_layered_does_not(rule):
    # flooding reads only the previous iteration's posteriors, so the order
    # of the check rows cannot matter (up to the order of the final sums);
    # the layered schedule depends on it
    g = make_graph(2, 16).sub(10)
    perm = np.random.default_rng(3).permutation(g.M)
    gp = _permute_rows(g, perm)
    b = make_batch(g, 8, 1.0, data_seed=13)
    lf = b.q.astype(np.float64) / 4
    kw = dict(rule=rule, max_iter=5, early_exit=False, want_llr=True)
    _, _, _, f0 = oracle.decode_bp(g, lf, schedule="flooding", **kw)
    _, _, _, f1 = oracle.decode_bp(gp, lf, schedule="flooding", **kw)
    assert np.allclose(f0, f1, rtol=1e-12, atol=1e-9)
    _, _, _, l0 = oracle.decode_bp(g, lf, schedule="layered", **kw)
    _, _, _, l1 = oracle.decode_bp(gp, lf, schedule="layered", **kw)
    assert np.abs(l0 - l1).max() > 1e-3
    assert np.abs(l0 - f0).max() > 1e-3
