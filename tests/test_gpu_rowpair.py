"""The int8 row-pair kernel (one codeword per Z/2 lanes, each lane updating
check rows u and u + Z/2 as the two halves of its packed registers) against
the CPU oracle, through the C ABI: bit-exact hard decisions, posteriors,
iteration counts and flags over lifts whose halves fill whole waves or not
(Z/2 = 8 .. 192), several codewords per workgroup with a ragged last
workgroup, the normalisation options, messages in device memory or in LDS,
and the same results as codeword pairs."""
import numpy as np
import pytest

from synth import make_batch

from test_gpu_parity import _graph, assert_i8_equal, gpu_decode, oracle_i8

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05534_amd import ldpc
    ldpc.lib()
    yield


@pytest.mark.parametrize("bg,Z,rows,n,cpw,ebn0", [
    (1, 384, 46, 3, 1, 1.5),
    (1, 384, 46, 5, 2, 1.25),   # two codewords per workgroup, ragged last one
    (2, 384, 42, 4, 1, 1.0),
    (1, 352, 46, 3, 1, 1.75),   # 176 lanes: the third wave is partly idle
    (2, 256, 30, 6, 3, 1.25),
    (1, 64, 46, 9, 6, 2.0),
    (1, 40, 46, 33, 16, 1.5),   # 20 lanes per codeword, 320 per workgroup
    (1, 24, 20, 17, 3, 1.5),
    (2, 16, 42, 40, 4, 1.5),
])
def test_rowpair_equals_oracle(bg, Z, rows, n, cpw, ebn0):
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=700 + Z + rows)
    print(f"[rowpair] bg={bg} Z={Z} rows={rows} n={n} cpw={cpw}", flush=True)
    got = gpu_decode(bg, Z, rows, b.q, pairing="rows", cw_per_block=cpw)
    assert_i8_equal(got, oracle_i8(g, b.q))


@pytest.mark.parametrize("opts", [
    dict(offset=2),
    dict(beta=1.0, offset=1),
    dict(max_iter=1),
    dict(max_iter=25),
    dict(early_exit=False),
])
def test_rowpair_options(opts):
    g = _graph(1, 128, 46)
    b = make_batch(g, 6, 1.25, data_seed=71)
    got = gpu_decode(1, 128, 46, b.q, pairing="rows", cw_per_block=2, **opts)
    assert_i8_equal(got, oracle_i8(g, b.q, **opts))


def test_rowpair_learned_weights():
    g = _graph(1, 384, 46)
    b = make_batch(g, 4, 1.0, data_seed=72)
    w = np.random.default_rng(3).integers(40, 140, (10, 46)).astype(np.uint8)
    got = gpu_decode(1, 384, 46, b.q, pairing="rows", weights=w)
    assert_i8_equal(got, oracle_i8(g, b.q, weights=w))


def test_rowpair_saturated_inputs():
    # every LLR -128 (read as -127) and every LLR +127: saturation on both sides
    g = _graph(2, 384, 42)
    for v in (-128, 127):
        q = np.full((2, g.T), v, np.int8)
        got = gpu_decode(2, 384, 42, q, pairing="rows", max_iter=4)
        assert_i8_equal(got, oracle_i8(g, q, max_iter=4))


@pytest.mark.parametrize("bg,rows,early_exit", [(1, 46, True), (1, 46, False), (2, 42, False)])
def test_auto_pairing_equals_codeword_pairs(bg, rows, early_exit):
    # small batches at Z = 384 take row pairs by default (BG2-shaped, whose
    # rows weigh at most 10 blocks: with the messages in LDS); results are
    # the same as codeword pairs and the oracle's
    g = _graph(bg, 384, rows)
    b = make_batch(g, 7, 1.5, data_seed=73)
    auto = gpu_decode(bg, 384, rows, b.q, early_exit=early_exit)
    cw = gpu_decode(bg, 384, rows, b.q, pairing="codewords", early_exit=early_exit)
    assert_i8_equal(auto, cw)
    assert_i8_equal(auto, oracle_i8(g, b.q, early_exit=early_exit))


@pytest.mark.parametrize("bg,Z,rows,n", [
    (1, 16, 46, 23),   # four codewords per workgroup by default, ragged end
    (1, 24, 46, 13),   # four: 48 of 64 lanes
    (2, 40, 42, 8),    # three: 60 of 64 lanes
    (2, 56, 30, 5),    # two: 56 of 64 lanes
    (1, 72, 46, 11),   # one: 36 of 64 lanes
    (2, 144, 42, 9),   # two: 144 lanes in three waves
    (1, 208, 46, 5),   # two: 208 lanes in four waves, ragged end
    (1, 320, 46, 3),   # one: 160 lanes in three waves
])
def test_rowpair_default_cpw_other_lifts(bg, Z, rows, n):
    # row pairs with the default codewords per workgroup; lifts that are
    # not powers of two leave partial waves
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, 1.5, data_seed=800 + Z)
    print(f"[rowpair default cpw] bg={bg} Z={Z} rows={rows} n={n}", flush=True)
    got = gpu_decode(bg, Z, rows, b.q, pairing="rows")
    assert_i8_equal(got, oracle_i8(g, b.q))
    assert_i8_equal(got, gpu_decode(bg, Z, rows, b.q, pairing="codewords"))


def test_auto_row_pairs_large_batch():
    # early exit at a small lift with more than four codewords per CU: the
    # default launch takes row pairs; same results as codeword pairs, and
    # the oracle's on a sample
    g = _graph(2, 16, 42)
    n = 4 * torch.cuda.get_device_properties(0).multi_processor_count + 37
    b = make_batch(g, n, 1.5, data_seed=830)
    print(f"[rowpair auto] BG2 Z=16 n={n}", flush=True)
    auto = gpu_decode(2, 16, 42, b.q)
    assert_i8_equal(auto, gpu_decode(2, 16, 42, b.q, pairing="codewords"))
    idx = np.random.default_rng(8).choice(n, 64, replace=False)
    assert_i8_equal(tuple(x[idx] for x in auto), oracle_i8(g, b.q[idx]))


@pytest.mark.parametrize("bg,Z,rows,n,cpw", [
    (1, 384, 46, 2, 1),    # one codeword's state: 147 kB of LDS
    (2, 384, 42, 3, 0),
    (1, 128, 46, 5, 2),    # ragged last workgroup
    (2, 64, 30, 9, 4),
    (1, 40, 46, 7, 3),     # partial wave
    (2, 16, 42, 11, 0),
])
def test_rowpair_lds_messages(bg, Z, rows, n, cpw):
    # messages in LDS after each codeword's posteriors: same results as
    # device-placed messages and as the oracle, with and without early exit
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, 1.5, data_seed=820 + Z)
    print(f"[rowpair lds] bg={bg} Z={Z} rows={rows} n={n} cpw={cpw}", flush=True)
    for ee in (True, False):
        got = gpu_decode(bg, Z, rows, b.q, pairing="rows", msg_placement="lds", cw_per_block=cpw,
                         early_exit=ee)
        assert_i8_equal(got, oracle_i8(g, b.q, early_exit=ee))
        assert_i8_equal(got, gpu_decode(bg, Z, rows, b.q, pairing="rows",
                                        msg_placement="device", cw_per_block=cpw, early_exit=ee))


def test_rowpair_noalloc():
    g = _graph(1, 384, 46)
    b = make_batch(g, 3, 1.5, data_seed=74)
    a = gpu_decode(1, 384, 46, b.q, pairing="rows")
    na = gpu_decode(1, 384, 46, b.q, pairing="rows", noalloc=True)
    assert_i8_equal(na, a)


def test_rowpair_refusals():
    from paper_2009_05534_amd import ldpc
    g = _graph(1, 64, 30)
    q = make_batch(g, 4, 1.5, data_seed=75).q
    for kw in (dict(pairing="rows", schedule="persistent"),
               dict(pairing="rows", lanes_per_row=2),
               dict(pairing="rows", precision="f16")):
        with pytest.raises(ldpc.LdpcError):
            gpu_decode(1, 64, 30, q, **kw)
    with pytest.raises(ValueError):
        gpu_decode(1, 64, 30, q, pairing="lanes")
