"""The allocation-free decode entry point (ldpc_decode_noalloc, messages in
the library's static per-device scratch) against ldpc_decode_ex, through the
C ABI: identical outputs on two calls in a row, the second smaller, in both
number formats and both message placements; sizes beyond the scratch and
graphs without resident device tables are refused without touching the
outputs."""
import numpy as np
import pytest

from synth import make_batch, make_graph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05534_amd import ldpc
    ldpc.lib()
    yield


def _both(bg, Z, rows, q, precision, **kw):
    """(decode_ex outputs, decode_noalloc outputs) of the same input."""
    from paper_2009_05534_amd import ldpc
    llr = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    outs = []
    for noalloc in (False, True):
        bits, iters, ok, post = ldpc.decode(llr, bg, Z, rows, precision=precision,
                                            want_llr=True, noalloc=noalloc, **kw)
        torch.cuda.synchronize()
        outs.append(tuple(t.cpu().numpy() for t in (bits, iters, ok, post)))
    return outs


def _same(a, b):
    for x, y, name in zip(a, b, ("bits", "iters", "ok", "posteriors")):
        assert x.shape == y.shape and x.dtype == y.dtype, name
        if x.dtype == np.float16:
            x, y = x.view(np.uint16), y.view(np.uint16)
        assert (x == y).all(), f"{name} differ"


@pytest.mark.parametrize("bg,Z,rows,precision,n1,n2,ebn0,kw", [
    # BG1 Z = 384, all rows: int8 messages in the scratch (device placement),
    # 300 then 37 codewords (odd: a pair with an idle partner)
    (1, 384, 46, "i8", 300, 37, 1.5, {}),
    # the same at a fixed 10 iterations (every message row written and read)
    (1, 384, 46, "i8", 120, 7, 1.25, {"early_exit": False}),
    # binary16: messages always in the scratch
    (1, 384, 46, "f16", 200, 9, 1.5, {}),
    # small lift whose messages fit LDS (no scratch used), and the same
    # forced to device placement
    (2, 16, 42, "i8", 500, 33, 2.0, {}),
    (2, 16, 42, "i8", 500, 33, 2.0, {"msg_placement": "device"}),
    (2, 64, 20, "f16", 64, 5, 1.5, {}),
])
def test_noalloc_equals_decode_ex(bg, Z, rows, precision, n1, n2, ebn0, kw):
    from paper_2009_05534_amd import ldpc
    g = make_graph(bg, Z)
    ldpc.register(g)
    sub = g.sub(rows) if rows != g.M else g
    # the graph's device tables are uploaded by an ordinary decode first
    warm = make_batch(sub, 2, ebn0, data_seed=70)
    ldpc.decode(torch.from_numpy(warm.q).cuda(), bg, Z, rows, precision=precision)
    torch.cuda.synchronize()
    for i, n in enumerate((n1, n2)):
        print(f"[noalloc] bg={bg} Z={Z} rows={rows} {precision} call {i + 1}: {n} codewords",
              flush=True)
        b = make_batch(sub, n, ebn0, data_seed=71 + i)
        ex, na = _both(bg, Z, rows, b.q, precision, **kw)
        _same(ex, na)


def test_noalloc_refuses_oversize_and_cold_graph():
    from paper_2009_05534_amd import ldpc
    g = make_graph(1, 384)
    ldpc.register(g)
    b = make_batch(g, 2, 1.5, data_seed=72)
    ldpc.decode(torch.from_numpy(b.q).cuda(), 1, 384, g.M)  # uploads the tables
    torch.cuda.synchronize()
    K, T, Nc, E = ldpc.query(1, 384, g.M)
    # n * E_pad * Z + 16 bytes of int8 messages with row pairs (the default
    # here: early exit), 2 * ceil(n/2) * E_pad * Z + 16 with codeword pairs:
    # 515 codewords need more than the 64 MiB scratch, 514 fit exactly
    n = 515
    llr = torch.zeros((n, T), dtype=torch.int8, device="cuda")
    bits = torch.full((n, K // 8), 0xA5, dtype=torch.uint8, device="cuda")
    iters = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(ldpc.LdpcError) as ei:
        ldpc.decode_into(llr, 1, 384, g.M, bits, iters, noalloc=True)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert (bits == 0xA5).all() and (iters == -7).all()
    # 514 codewords fit exactly
    ldpc.decode_into(llr[:514], 1, 384, g.M, bits[:514], iters[:514], noalloc=True)
    torch.cuda.synchronize()
    assert (iters[:514] == 1).all()  # all-zero LLRs: every check holds after one iteration
    # a freshly registered graph has no device tables until an ordinary decode
    g2 = make_graph(2, 24)
    ldpc.register(g2)
    K2, T2, _, _ = ldpc.query(2, 24, g2.M)
    llr2 = torch.zeros((4, T2), dtype=torch.int8, device="cuda")
    bits2 = torch.empty((4, K2 // 8), dtype=torch.uint8, device="cuda")
    iters2 = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(ldpc.LdpcError) as ei:
        ldpc.decode_into(llr2, 2, 24, g2.M, bits2, iters2, noalloc=True)
    assert ei.value.code == -4
    ldpc.decode_into(llr2, 2, 24, g2.M, bits2, iters2)
    ldpc.decode_into(llr2, 2, 24, g2.M, bits2, iters2, noalloc=True)
    torch.cuda.synchronize()
    assert (iters2 == 1).all()
