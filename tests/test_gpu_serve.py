"""Continuous-batching server: every block's result in the mix equals
decoding that block alone with the same policy (int8: bit-exact), and the
server reports latency and deadline statistics."""
import numpy as np
import pytest

from synth import LIFTS, make_graph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def server_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05534_amd import ldpc, serve
    for bg in (1, 2):
        for Z in LIFTS:
            ldpc.register(make_graph(bg, Z))
    return serve


@pytest.mark.parametrize("rate", [2e3, 5e4])
def test_mix_equals_alone(server_mod, rate):
    serve = server_mod
    blocks = serve.make_trace(120, seed=6)
    rng = np.random.default_rng(0)
    wq = rng.integers(80, 112, (10, 46)).astype(np.uint8)
    srv = serve.Server(weights_bg1=wq, n_slots=4, mem_budget=64 << 20)
    trace = serve.rescale(blocks, rate)
    stats = srv.run(trace)
    assert stats["blocks"] == 120 and stats["latency_ms_p99"] > 0
    assert 0.0 <= stats["deadline_met"] <= 1.0
    for b in trace:
        bits, iters, ok = srv.decode_alone(b)
        assert (b.bits == bits).all(), b.id
        assert (b.iters == iters).all(), b.id
        assert (b.ok == ok).all(), b.id


def test_memory_budget_limits_admission(server_mod):
    serve = server_mod
    blocks = serve.rescale(serve.make_trace(40, seed=7), 1e6)  # all arrive at once
    big = max(serve.message_bytes(b.bg, b.Z, b.rows, b.n_cw) for b in blocks)
    srv = serve.Server(n_slots=8, mem_budget=big)  # one block's worth at a time
    stats = srv.run(blocks)
    # admission never let the messages in flight exceed the budget, so the
    # blocks needed at least total/budget launches
    total = sum(serve.message_bytes(b.bg, b.Z, b.rows, b.n_cw) for b in blocks)
    assert 0 < stats["peak_message_bytes"] <= big
    assert stats["launches"] >= -(-total // big)
    srv2 = serve.Server(n_slots=1, mem_budget=1)
    with pytest.raises(ValueError):
        srv2.run(serve.rescale(serve.make_trace(3, seed=8), 1e3))
