"""The low-latency int8 mapping (alpha = 2 or 4 lanes per check row, chunk
minima merged through LDS; §IV) against the CPU oracle, through the C ABI:
bit-exact hard decisions, final posteriors, iteration counts and success
flags on the listed shapes, options, per-row weights, seeded random shapes
and packings, plus the argument checks."""
import math

import numpy as np
import pytest

from synth import make_batch

from test_gpu_parity import CASES, _graph, assert_i8_equal, gpu_decode, oracle_i8

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05534_amd import ldpc
    ldpc.lib()
    yield


def _fits(alpha, Z, pairs=None):
    """alpha * P * Z lanes in one workgroup, P * Z whole waves."""
    if pairs is None:
        pairs = 64 // math.gcd(Z, 64)
    return (pairs * Z) % 64 == 0 and alpha * pairs * Z <= 1024


@pytest.mark.parametrize("alpha", [2, 4])
@pytest.mark.parametrize("bg,Z,rows,n,ebn0", CASES)
def test_ll_bit_exact(alpha, bg, Z, rows, n, ebn0):
    from paper_2009_05534_amd import ldpc
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=300 + Z + rows)
    print(f"[ll] alpha={alpha} bg={bg} Z={Z} rows={rows} n={n}", flush=True)
    if not _fits(alpha, Z):
        with pytest.raises(ldpc.LdpcError):
            gpu_decode(bg, Z, rows, b.q, lanes_per_row=alpha)
        return
    assert_i8_equal(gpu_decode(bg, Z, rows, b.q, lanes_per_row=alpha), oracle_i8(g, b.q))


@pytest.mark.parametrize("alpha", [2, 4])
@pytest.mark.parametrize("opts", [
    dict(early_exit=False),
    dict(max_iter=1),
    dict(max_iter=25),
    dict(offset=2),
    dict(beta=1.0, offset=1, early_exit=False, max_iter=4),
])
def test_ll_options(alpha, opts):
    g = _graph(1, 64, 30)
    b = make_batch(g, 40, 1.25, data_seed=17)
    assert_i8_equal(gpu_decode(1, 64, 30, b.q, lanes_per_row=alpha, **opts),
                    oracle_i8(g, b.q, **opts))


@pytest.mark.parametrize("alpha", [2, 4])
def test_ll_per_iteration_row_weights(alpha):
    g = _graph(2, 96, 25)
    b = make_batch(g, 30, 1.5, data_seed=18)
    w = np.random.default_rng(10).integers(0, 256, (3, 25)).astype(np.uint8)
    got = gpu_decode(2, 96, 25, b.q, weights=w, max_iter=8, lanes_per_row=alpha)
    assert_i8_equal(got, oracle_i8(g, b.q, weights=w, max_iter=8))


@pytest.mark.parametrize("early_exit", [True, False])
def test_ll_full_size_sampled(early_exit):
    # BG1-shaped Z = 384, all 46 rows (core rows of 19 blocks: chunks of 10
    # and 9), 512 codewords; the oracle checks a sample
    g = _graph(1, 384, 46)
    b = make_batch(g, 512, 1.5, data_seed=19)
    got = gpu_decode(1, 384, 46, b.q, early_exit=early_exit, lanes_per_row=2)
    idx = np.random.default_rng(5).choice(512, 24, replace=False)
    assert_i8_equal(tuple(x[idx] for x in got), oracle_i8(g, b.q[idx], early_exit=early_exit))


def test_ll_single_codeword_and_degenerate():
    from synth import encode, noiseless_q
    g = _graph(1, 128, 46)
    u = np.random.default_rng(6).integers(0, 2, (3, g.K), dtype=np.uint8)
    for q in (noiseless_q(encode(g, u), g)[:1], np.full((1, g.T), -128, np.int8),
              np.zeros((2, g.T), np.int8), make_batch(g, 1, 1.0, data_seed=20).q):
        for alpha in (2, 4):
            assert_i8_equal(gpu_decode(1, 128, 46, q, lanes_per_row=alpha), oracle_i8(g, q))


def test_ll_packings_agree():
    # several pairs per workgroup (whole waves per chunk group) give the same
    # results as one
    g = _graph(2, 32, 42)
    b = make_batch(g, 61, 1.5, data_seed=21)
    ref = oracle_i8(g, b.q)
    for alpha, cpw in ((2, 4), (2, 8), (2, 16), (4, 4), (4, 8)):
        assert_i8_equal(gpu_decode(2, 32, 42, b.q, lanes_per_row=alpha, cw_per_block=cpw), ref)


def test_ll_refusals():
    from paper_2009_05534_amd import ldpc
    g = _graph(1, 384, 46)
    q = make_batch(g, 2, 1.5, data_seed=22).q
    for kw in (dict(lanes_per_row=4),                       # 4 * 384 lanes > 1024
               dict(lanes_per_row=3),                       # not 1, 2 or 4
               dict(lanes_per_row=2, msg_placement="lds"),  # device messages only
               dict(lanes_per_row=2, precision="f16"),      # int8 only
               dict(lanes_per_row=2, cw_per_block=4)):      # 2 * 2 * 384 lanes > 1024
        with pytest.raises(ldpc.LdpcError):
            gpu_decode(1, 384, 46, q, **kw)
    g2 = _graph(2, 24, 42)
    q2 = make_batch(g2, 2, 1.5, data_seed=23).q
    with pytest.raises(ldpc.LdpcError):                     # 2 pairs * 24 lanes: not whole waves
        gpu_decode(2, 24, 42, q2, lanes_per_row=2, cw_per_block=4)


def _random_cases(n_cases, seed):
    import random
    rng = random.Random(seed)
    cases = []
    while len(cases) < n_cases:
        bg = rng.choice([1, 2])
        Z = 8 * rng.randint(1, 48)
        rows = rng.randint(4, 46 if bg == 1 else 42)
        alpha = rng.choice([2, 4])
        base = 64 // math.gcd(Z, 64)
        pairs = base * rng.choice([1, 1, 2])
        if not _fits(alpha, Z, pairs):
            continue
        n = rng.randint(1, 40 if Z <= 192 else 12)
        cases.append((len(cases), bg, Z, rows, n, rng.uniform(0.5, 3.0), rng.random() < 0.7,
                      alpha, 2 * pairs))
    return cases


@pytest.mark.parametrize("i,bg,Z,rows,n,ebn0,ee,alpha,cpw", _random_cases(30, 20261204))
def test_ll_random_shapes(i, bg, Z, rows, n, ebn0, ee, alpha, cpw):
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=3000 + i)
    print(f"[ll] case {i}: bg={bg} Z={Z} rows={rows} n={n} alpha={alpha} cpw={cpw}", flush=True)
    got = gpu_decode(bg, Z, rows, b.q, early_exit=ee, lanes_per_row=alpha, cw_per_block=cpw)
    assert_i8_equal(got, oracle_i8(g, b.q, early_exit=ee))
