"""ldpc_tune: the launch-configuration autotuner times the int8 candidates
(lanes per check row, codeword pairs per workgroup, message placement,
schedule) on a shape and batch size, and later default-knob calls of that
shape take the fastest. Every candidate and the tuned default call give the oracle's
results bit for bit."""
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


@pytest.mark.parametrize("bg,Z,rows,n", [(2, 32, 42, 37), (1, 128, 46, 64), (2, 384, 42, 6)])
def test_tune_then_default_equals_oracle(bg, Z, rows, n):
    from paper_2009_05534_amd import ldpc
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, 1.5, data_seed=400 + Z)
    print(f"[tune] bg={bg} Z={Z} rows={rows} n={n}", flush=True)
    llr = torch.from_numpy(b.q).cuda()
    K = g.K
    bits = torch.zeros((n, (K + 7) // 8), dtype=torch.uint8, device="cuda")
    iters = torch.zeros(n, dtype=torch.int32, device="cuda")
    ok = torch.zeros(n, dtype=torch.uint8, device="cuda")
    choice = ldpc.decode_into(llr, bg, Z, rows, bits, iters, out_ok=ok, tune=True)
    torch.cuda.synchronize()
    assert choice["candidates"] >= 2 and choice["ms"] > 0, choice
    assert choice["lanes_per_row"] in (1, 2, 4), choice
    assert choice["schedule"] in ("static", "persistent"), choice
    assert choice["msg_placement"] in ("auto", "lds", "device"), choice
    ref = oracle_i8(g, b.q)
    # the tuner's own outputs (those of its last candidate)
    assert_i8_equal((bits.cpu().numpy(), iters.cpu().numpy(), ok.cpu().numpy()),
                    ref[:3])
    # the next default call takes the tuned configuration
    assert_i8_equal(gpu_decode(bg, Z, rows, b.q), ref)
    # and the chosen knobs spelled out give the same
    assert choice["pairing"] in ("auto", "codewords", "rows"), choice
    kw = dict(lanes_per_row=choice["lanes_per_row"], cw_per_block=choice["cw_per_block"],
              msg_placement=choice["msg_placement"], schedule=choice["schedule"],
              pairing=choice["pairing"])
    assert_i8_equal(gpu_decode(bg, Z, rows, b.q, **kw), ref)


def test_tune_refusals():
    from paper_2009_05534_amd import ldpc
    g = _graph(1, 64, 30)
    q = torch.from_numpy(make_batch(g, 4, 1.5, data_seed=401).q).cuda()
    bits = torch.zeros((4, (g.K + 7) // 8), dtype=torch.uint8, device="cuda")
    iters = torch.zeros(4, dtype=torch.int32, device="cuda")
    for kw in (dict(cw_per_block=2), dict(lanes_per_row=2), dict(msg_placement="lds"),
               dict(precision="f16"), dict(schedule="persistent"), dict(max_workgroups=2),
               dict(pairing="rows")):
        with pytest.raises(ldpc.LdpcError):
            ldpc.decode_into(q, 1, 64, 30, bits, iters, tune=True, **kw)
