"""GPU decoder (C ABI through the Python binding) against the CPU oracle on
the same seeded inputs.

int8: bit-exact hard decisions, final posteriors, iteration counts and
success flags. binary16: identical hard decisions, iteration counts and
flags; the contract for posteriors is 1e-2 relative error (denominator
max(|ref|, 1)), and since both sides round every operation to binary16
(nearest, ties to even) in the same order, the posteriors are also
required to be bit-identical.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from libgraph import library_graph
from synth import encode, make_batch, make_graph, noiseless_q

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F16_RTOL = 1e-2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05534_amd import ldpc
    ldpc.lib()
    yield


_registered = set()


def _graph(bg, Z, rows):
    """The seeded graph (bg, Z) registered with the library, as read back
    from it (ldpc_get_graph): the oracle decodes the library's table."""
    from paper_2009_05534_amd import ldpc
    if (bg, Z) not in _registered:
        ldpc.register(make_graph(bg, Z))
        _registered.add((bg, Z))
    return library_graph(bg, Z, rows)


def gpu_decode(bg, Z, rows, q, precision="i8", weights=None, **kw):
    from paper_2009_05534_amd import ldpc
    llr = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    w = None
    if weights is not None:
        w = torch.from_numpy(np.ascontiguousarray(weights)).cuda()
    bits, iters, ok, out = ldpc.decode(llr, bg, Z, rows, precision=precision, weights=w,
                                       want_llr=True, **kw)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), iters.cpu().numpy(), ok.cpu().numpy(), out.cpu().numpy()


def oracle_i8(g, q, **kw):
    kw2 = dict(kw)
    if "beta" in kw2:
        b = kw2.pop("beta")
        kw2["wq"] = np.full((1, g.M), int(round(b * 128)), np.uint8)
    if "weights" in kw2:
        kw2["wq"] = kw2.pop("weights")
    if "offset" in kw2:
        kw2["delta"] = kw2.pop("offset")
    kw2.pop("cw_per_block", None)
    return oracle.decode_i8(g, q, want_llr=True, n_threads=8, **kw2)


def oracle_f16(g, q, **kw):
    kw2 = dict(kw)
    if "weights" in kw2:
        kw2["wh"] = kw2.pop("weights").view(np.uint16)
    if "offset" in kw2:
        kw2["delta"] = kw2.pop("offset")
    kw2.pop("cw_per_block", None)
    return oracle.decode_f16(g, q, want_llr=True, n_threads=8, **kw2)


def assert_i8_equal(got, ref):
    for name, a, b in zip(("bits", "iters", "ok", "llr"), got, ref):
        assert a.shape == b.shape, name
        bad = np.argwhere(a != b)
        assert bad.size == 0, f"{name} differs at {bad[:5].tolist()} ({len(bad)} entries)"


def assert_f16_close(got, ref):
    for name, a, b in zip(("bits", "iters", "ok"), got[:3], ref[:3]):
        bad = np.argwhere(a != b)
        assert bad.size == 0, f"{name} differs at {bad[:5].tolist()} ({len(bad)} entries)"
    a = got[3].view(np.float16).astype(np.float64)
    b = oracle.f16_to_f64(ref[3])
    rel = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    assert rel.max() <= F16_RTOL, f"max rel err {rel.max()}"
    bad = np.argwhere(got[3].view(np.uint16) != ref[3])
    assert bad.size == 0, f"binary16 posteriors differ at {bad[:5].tolist()} ({len(bad)} entries)"
    # hard decisions of every variable, not only the information bits
    assert ((a < 0) == (b < 0)).all()


CASES = [
    # bg, Z, rows, n_cw, Eb/N0
    (2, 16, 42, 1000, 2.0),   # the small BG2-shaped workload, all 1000 codewords
    (1, 16, 46, 37, 1.0),
    (1, 32, 10, 64, 1.5),
    (2, 64, 20, 50, 1.0),
    (1, 96, 46, 21, 1.5),
    (2, 128, 4, 40, 3.0),
    (1, 192, 30, 13, 1.5),
    (2, 256, 42, 9, 1.0),
    (1, 384, 46, 8, 1.5),
    (1, 384, 5, 11, 2.0),
]


@pytest.mark.parametrize("bg,Z,rows,n,ebn0", CASES)
def test_i8_bit_exact(bg, Z, rows, n, ebn0):
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=100 + Z + rows)
    assert_i8_equal(gpu_decode(bg, Z, rows, b.q), oracle_i8(g, b.q))


@pytest.mark.parametrize("bg,Z,rows,n,ebn0", [c for c in CASES if c[3] <= 64])
def test_f16_matches(bg, Z, rows, n, ebn0):
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=200 + Z + rows)
    assert_f16_close(gpu_decode(bg, Z, rows, b.q, precision="f16"), oracle_f16(g, b.q))


@pytest.mark.parametrize("opts", [
    dict(early_exit=False),
    dict(max_iter=1),
    dict(max_iter=25),
    dict(offset=2),
    dict(beta=0.875),
    dict(beta=1.0, offset=1, early_exit=False, max_iter=4),
])
def test_i8_options(opts):
    g = _graph(1, 64, 30)
    b = make_batch(g, 40, 1.25, data_seed=7)
    assert_i8_equal(gpu_decode(1, 64, 30, b.q, **opts), oracle_i8(g, b.q, **opts))


def test_i8_per_iteration_row_weights():
    g = _graph(2, 96, 25)
    b = make_batch(g, 30, 1.5, data_seed=8)
    w = np.random.default_rng(0).integers(0, 256, (3, 25)).astype(np.uint8)
    got = gpu_decode(2, 96, 25, b.q, weights=w, max_iter=8)
    assert_i8_equal(got, oracle_i8(g, b.q, weights=w, max_iter=8))


def test_f16_options_and_weights():
    g = _graph(1, 128, 20)
    b = make_batch(g, 24, 1.5, data_seed=9)
    for opts in (dict(early_exit=False), dict(offset=0.5), dict(beta=0.8125)):
        assert_f16_close(gpu_decode(1, 128, 20, b.q, precision="f16", **opts),
                         oracle_f16(g, b.q, **opts))
    w = np.random.default_rng(1).uniform(0.5, 1.0, (4, 20)).astype(np.float16)
    assert_f16_close(gpu_decode(1, 128, 20, b.q, precision="f16", weights=w, max_iter=7),
                     oracle_f16(g, b.q, weights=w, max_iter=7))


@pytest.mark.parametrize("precision", ["i8", "f16"])
def test_workgroup_packing_does_not_change_results(precision):
    # Different codewords-per-workgroup packings and a shuffled batch order
    # give the same per-codeword results (a missing barrier or a slot
    # mix-up shows up here).
    g = _graph(2, 32, 42)
    b = make_batch(g, 61, 1.5, data_seed=10)
    ref = gpu_decode(2, 32, 42, b.q, precision=precision)
    for cpw in (1, 3, 7):
        got = gpu_decode(2, 32, 42, b.q, precision=precision, cw_per_block=cpw)
        for a, r in zip(got, ref):
            assert (a == r).all()
    perm = np.random.default_rng(2).permutation(61)
    got = gpu_decode(2, 32, 42, b.q[perm], precision=precision)
    for a, r in zip(got, ref):
        assert (a == r[perm]).all()


@pytest.mark.parametrize("precision", ["i8", "f16"])
def test_degenerate_inputs(precision):
    g = _graph(1, 32, 12)
    u = np.random.default_rng(3).integers(0, 2, (5, g.K), dtype=np.uint8)
    c = encode(g, u)
    cases = [
        noiseless_q(c, g),                                   # one iteration
        np.full((3, g.T), -128, np.int8),                    # saturated, -128 read as -127
        np.zeros((4, g.T), np.int8),                         # no information at all
        np.full((1, g.T), 127, np.int8),                     # single codeword
    ]
    for q in cases:
        got = gpu_decode(1, 32, 12, q, precision=precision)
        ref = (oracle_i8 if precision == "i8" else oracle_f16)(g, q)
        (assert_i8_equal if precision == "i8" else assert_f16_close)(got, ref)
    got = gpu_decode(1, 32, 12, cases[0], precision=precision)
    assert (got[1] == 1).all() and got[2].all()
    assert (oracle.unpack_bits(got[0], g.K) == u).all()


@pytest.mark.parametrize("early_exit", [True, False])
def test_full_size_sampled(early_exit):
    # BG1-shaped Z=384, all 46 rows, 4096 codewords in one call with the
    # default launch configuration (early exit, and the fixed 10 iterations
    # of the benchmark's roofline run); the oracle checks a sample of them.
    g = _graph(1, 384, 46)
    n = 4096
    b = make_batch(g, n, 1.5, data_seed=5)
    got = gpu_decode(1, 384, 46, b.q, early_exit=early_exit)
    idx = np.random.default_rng(4).choice(n, 48, replace=False)
    ref = oracle_i8(g, b.q[idx], early_exit=early_exit)
    assert_i8_equal(tuple(x[idx] for x in got), ref)
    if not early_exit:
        return
    got16 = gpu_decode(1, 384, 46, b.q[:512], precision="f16")
    idx16 = idx[idx < 512][:16]
    ref16 = oracle_f16(g, b.q[idx16])
    assert_f16_close(tuple(x[idx16] for x in got16), ref16)


@pytest.mark.parametrize("bg,Z,rows", [(1, 384, 46), (2, 64, 42), (1, 16, 20), (1, 192, 8)])
def test_i8_message_placements_agree(bg, Z, rows):
    # Messages kept in LDS or streamed through device memory: same results,
    # both equal to the oracle.
    g = _graph(bg, Z, rows)
    b = make_batch(g, 12, 1.5, data_seed=11 + Z)
    ref = oracle_i8(g, b.q)
    from paper_2009_05534_amd import ldpc
    # LDS placement holds a codeword pair's posteriors and messages in one
    # workgroup: 2 * (N + E) * Z bytes, more than a CU has for the full BG1
    # graph at Z = 384, where it is refused.
    K, T, Nc, E = ldpc.query(bg, Z, rows)
    fits = 2 * (Nc // Z + E) * Z + 8 <= 160 * 1024
    for placement in ("lds", "device"):
        for cpw in (0, 1, 3):
            if placement == "lds" and not fits:
                with pytest.raises(ldpc.LdpcError):
                    gpu_decode(bg, Z, rows, b.q, msg_placement=placement, cw_per_block=cpw)
                continue
            got = gpu_decode(bg, Z, rows, b.q, msg_placement=placement, cw_per_block=cpw)
            assert_i8_equal(got, ref)


def _wide_graph(Z, weights, kb, seed):
    """Random base graph with the given row weights (columns and shifts from
    the seed), registered as (bg=1, Z) with a lift the other tests do not
    use. Rows wider than 10 blocks other than 19 take the decoder's
    bound-weight path; weights above 20 its widest kernel."""
    from synth import make_toy_graph
    from paper_2009_05534_amd import ldpc
    rng = np.random.default_rng(seed)
    M, N = len(weights), kb + len(weights)
    base = -np.ones((M, N), np.int64)
    for r, w in enumerate(weights):
        # row r may use the information columns and parity columns up to its
        # own (the core rows share the first four): nested sub-codes
        n_avail = kb + max(r + 1, 4)
        base[r, rng.choice(n_avail, size=w, replace=False)] = rng.integers(0, Z, size=w)
    g = dataclasses.replace(make_toy_graph(base, Z, kb, n_punct=2), bg=1)
    ldpc.register(g)
    _registered.discard((1, Z))  # (1, Z) now holds this graph, not the seeded one
    return library_graph(1, Z)


@pytest.mark.parametrize("Z,weights,kb", [
    (40, [11, 12, 13, 14, 15, 16, 17, 18, 20, 19, 3, 10], 20),
    (24, [21, 25, 32, 8, 30, 2], 28),
])
def test_i8_wide_rows(Z, weights, kb):
    g = _wide_graph(Z, weights, kb, seed=Z)
    rng = np.random.default_rng(Z + 1)
    # random channel values (no codeword: run to the iteration limit) and,
    # in the first codewords, noisy observations of the all-zero codeword
    # (a codeword of every graph), which settle after a few iterations
    q = np.clip(rng.normal(0, 40, (13, g.T)), -128, 127).astype(np.int8)
    mean = np.array([25, 30, 40, 50, 60])[:, None]
    q[:5] = np.clip(rng.normal(mean, 16, (5, g.T)), -128, 127).astype(np.int8)
    for placement in ("lds", "device"):
        for early in (True, False):
            ref = oracle_i8(g, q, early_exit=early)
            got = gpu_decode(1, Z, g.M, q, msg_placement=placement, early_exit=early)
            assert_i8_equal(got, ref)


def _random_cases(n_cases, seed):
    import random
    rng = random.Random(seed)
    cases = []
    for i in range(n_cases):
        bg = rng.choice([1, 2])
        Z = 8 * rng.randint(1, 48)           # any supported lift, not only the listed ones
        rows = rng.randint(4, 46 if bg == 1 else 42)
        n = rng.randint(1, 40 if Z <= 192 else 12)
        cases.append((i, bg, Z, rows, n, rng.uniform(0.5, 3.0), rng.random() < 0.7,
                      rng.choice(["auto", "device", "lds"]), rng.choice([0, 2, 4])))
    return cases


@pytest.mark.parametrize("i,bg,Z,rows,n,ebn0,ee,placement,cpw", _random_cases(40, 20261203))
def test_random_shapes(i, bg, Z, rows, n, ebn0, ee, placement, cpw):
    """Seeded random shapes, lifts, batch sizes, message placements and
    workgroup packings: int8 bit-exact, binary16 close (small batches)."""
    from paper_2009_05534_amd import ldpc
    g = _graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=2000 + i)
    try:
        got = gpu_decode(bg, Z, rows, b.q, early_exit=ee, msg_placement=placement,
                         cw_per_block=cpw)
    except ldpc.LdpcError:
        # LDS placement of a pair that does not fit a workgroup is refused
        assert placement == "lds"
        return
    assert_i8_equal(got, oracle_i8(g, b.q, early_exit=ee))
    if n <= 16:
        gf = gpu_decode(bg, Z, rows, b.q, precision="f16", early_exit=ee)
        assert_f16_close(gf, oracle_f16(g, b.q, early_exit=ee))
