"""The persistent int8 schedule (opt-in: codeword pairs take the next
codeword as soon as one of theirs finishes) against the CPU oracle, through
the C ABI:
few workgroups over many codewords, so that every half of every pair is
refilled several times with codewords that need different iteration
counts; bit-exact hard decisions, posteriors, iteration counts and flags,
and the same results as the static schedule."""
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


@pytest.mark.parametrize("bg,Z,rows,n,mw,ebn0", [
    (1, 64, 46, 150, 1, 1.5),
    (2, 96, 42, 77, 2, 1.25),
    (1, 128, 30, 61, 1, 2.0),
    (2, 16, 42, 300, 1, 1.0),
    (1, 384, 46, 14, 1, 1.5),
    (1, 192, 46, 40, 3, 1.75),
])
def test_refill_equals_oracle(bg, Z, rows, n, mw, ebn0):
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=500 + Z + rows)
    print(f"[refill] bg={bg} Z={Z} rows={rows} n={n} workgroups<={mw}", flush=True)
    got = gpu_decode(bg, Z, rows, b.q, schedule="persistent", max_workgroups=mw)
    ref = oracle_i8(g, b.q)
    assert len(set(ref[1].tolist())) > 1  # codewords finish at different iterations
    assert_i8_equal(got, ref)


@pytest.mark.parametrize("opts", [
    dict(offset=2),
    dict(max_iter=1),
    dict(max_iter=25),
    dict(beta=1.0, offset=1),
])
def test_refill_options(opts):
    g = _graph(1, 64, 30)
    b = make_batch(g, 90, 1.25, data_seed=17)
    got = gpu_decode(1, 64, 30, b.q, schedule="persistent", max_workgroups=1, **opts)
    assert_i8_equal(got, oracle_i8(g, b.q, **opts))


def test_refill_equals_static_full_grid():
    g = _graph(1, 384, 46)
    b = make_batch(g, 700, 1.75, data_seed=31)
    a = gpu_decode(1, 384, 46, b.q, schedule="persistent")
    s = gpu_decode(1, 384, 46, b.q)
    assert_i8_equal(a, s)
    idx = np.random.default_rng(7).choice(700, 16, replace=False)
    assert_i8_equal(tuple(x[idx] for x in a), oracle_i8(g, b.q[idx]))


def test_refill_small_batches():
    # fewer codewords than one workgroup holds
    g = _graph(2, 96, 42)
    for n in (1, 3):
        b = make_batch(g, n, 1.5, data_seed=40 + n)
        assert_i8_equal(gpu_decode(2, 96, 42, b.q, schedule="persistent", max_workgroups=1),
                        oracle_i8(g, b.q))


def test_schedule_refusals():
    from paper_2009_05534_amd import ldpc
    g = _graph(1, 64, 30)
    q = make_batch(g, 4, 1.5, data_seed=45).q
    w = np.full((2, 30), 96, np.uint8)
    for kw in (dict(max_workgroups=-1),
               dict(schedule="persistent", msg_placement="lds"),
               dict(schedule="persistent", early_exit=False),
               dict(schedule="persistent", weights=w),
               dict(schedule="persistent", cw_per_block=4),
               dict(schedule="persistent", lanes_per_row=2),
               dict(schedule="persistent", noalloc=True)):
        with pytest.raises(ldpc.LdpcError):
            gpu_decode(1, 64, 30, q, **kw)
    with pytest.raises(ValueError):
        gpu_decode(1, 64, 30, q, schedule="dynamic")
