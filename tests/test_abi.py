"""The C-ABI library loads and exports every function include/ldpc.h
declares; argument checks reject bad input without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldpc.h")
LIB = os.path.join(ROOT, "paper_2009_05534_amd", "libldpc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2009_05534_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "ldpc_decode" in names and "ldpc_decode_ex" in names
    for n in names:
        assert hasattr(lib, n), n
    from paper_2009_05534_amd import ldpc
    assert set(ldpc.EXPORTS) == set(names)


def test_args_struct_layout(lib):
    from paper_2009_05534_amd import ldpc
    a = ldpc.Args()
    ldpc.lib().ldpc_args_init(ctypes.byref(a))
    assert (a.precision, a.max_iter, a.early_exit, a.beta_q, a.beta_h) == (0, 10, 1, 96, 0x3A00)


def test_graph_registration_checks(lib):
    from paper_2009_05534_amd import ldpc
    from synth import make_graph
    g = make_graph(1, 384)
    ldpc.register(g)
    assert ldpc.query(1, 384, 46) == (8448, 25344, 26112, 316)
    assert ldpc.query(1, 384, 4) == (8448, 24 * 384, 26 * 384, 76)
    with pytest.raises(ldpc.LdpcError):
        ldpc.query(1, 384, 3)
    with pytest.raises(ldpc.LdpcError):
        ldpc.query(2, 24, 10)  # nothing registered
    bad = g.shift.copy()
    bad[5] = 384
    with pytest.raises(ldpc.LdpcError):
        ldpc.set_graph(1, 384, g.M, g.kb, g.row_ptr, g.col, bad)
    with pytest.raises(ldpc.LdpcError):  # Z not a multiple of 8
        ldpc.set_graph(1, 12, g.M, g.kb, g.row_ptr, g.col, g.shift % 12)
    unsorted = g.col.copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    with pytest.raises(ldpc.LdpcError):
        ldpc.set_graph(1, 384, g.M, g.kb, g.row_ptr, unsorted, g.shift)


def test_decode_rejects_bad_arguments_before_launch(lib):
    from paper_2009_05534_amd import ldpc
    from synth import make_graph
    ldpc.register(make_graph(1, 384))  # the checks below reach past the graph lookup
    a = ldpc.Args()
    lib_ = ldpc.lib()
    lib_.ldpc_args_init(ctypes.byref(a))
    a.bg, a.Z, a.rows, a.n_cw = 1, 384, 46, 1
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -1  # null pointers
    a.llr_in = a.out_bits = a.out_iters = 16  # never dereferenced: checks fail first
    a.max_iter = 0
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -1
    a.max_iter = 10
    a.rows = 47
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -1
    a.rows = 46
    a.llr_in = 17  # the LLRs are read as 32-bit words: 4-byte alignment
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -1
    a.llr_in = 16
    a.pairing = 3  # not a pairing
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -1
    a.pairing, a.precision = 2, 1  # row pairs are int8 only
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -1
    a.pairing, a.precision = 0, 0
    job = ldpc.Job(bg=1, Z=384, rows=46, n_cw=1, llr=17, out_bits=16, out_iters=16)
    nb = ctypes.c_size_t()
    assert lib_.ldpc_decode_batch_bytes(ctypes.byref(job), 1, ctypes.byref(nb)) == -1
    job.llr = 16  # passes the checks (without a GPU the device tables then fail)
    assert lib_.ldpc_decode_batch_bytes(ctypes.byref(job), 1, ctypes.byref(nb)) in (0, -3)
    a.bg = 7
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -4
    assert lib_.ldpc_strerror(-4) == b"no graph registered for (bg, Z)"


# 64-bit FNV-1a digests of the seeded BG-shaped graphs as registered (the
# serialisation ldpc_graph_digest documents). A change of the generator, of
# its seed or of the registration shows up here without a GPU.
GRAPH_DIGESTS = {
    (1, 16): 0xfa3e352ac64691f6, (1, 32): 0x04781dd60869e805, (1, 64): 0x12bb92c0e39589f7,
    (1, 96): 0x41c5b9a7810d7709, (1, 128): 0x67d9d517a853400b, (1, 192): 0xf3e01120b1f0731d,
    (1, 256): 0xa42ed78e52ae34a4, (1, 384): 0xd9b4ecb517ac63f7,
    (2, 16): 0xb456a0fae817d9b4, (2, 32): 0x62eabcbdbc688626, (2, 64): 0x4410fcd8fa721a9e,
    (2, 96): 0x5e010df5469887f5, (2, 128): 0x7be67e2e0d1d5dd2, (2, 192): 0xcd7a794444470530,
    (2, 256): 0x058183d5c1e6d741, (2, 384): 0xce829705b36186da,
}


def _fnv1a64_words(words):
    """FNV-1a 64 over little-endian 32-bit words (the published constants)."""
    h = 0xcbf29ce484222325
    for w in words:
        for byte in int(w & 0xFFFFFFFF).to_bytes(4, "little"):
            h = ((h ^ byte) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_graph_digest_and_readback(lib):
    from paper_2009_05534_amd import ldpc
    from synth import LIFTS, make_graph
    for bg in (1, 2):
        for Z in LIFTS:
            g = make_graph(bg, Z)
            ldpc.register(g)
            # called through the raw C ABI
            out = ctypes.c_uint64()
            assert lib.ldpc_graph_digest(bg, Z, ctypes.byref(out)) == 0
            assert out.value == GRAPH_DIGESTS[(bg, Z)], (bg, Z, hex(out.value))
            words = [bg, Z, g.M, g.kb, *g.row_ptr.tolist(), *g.col.tolist(), *g.shift.tolist()]
            assert out.value == _fnv1a64_words(words)
            m, kb, nnz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(0)
            assert lib.ldpc_get_graph(bg, Z, ctypes.byref(m), ctypes.byref(kb),
                                      ctypes.byref(nnz), None, None, None) == 0
            assert (m.value, kb.value, nnz.value) == (g.M, g.kb, g.E)
            row, col, sh = (np.full(g.E, -1, np.int16) for _ in range(3))
            assert lib.ldpc_get_graph(bg, Z, None, None, ctypes.byref(nnz),
                                      row.ctypes.data_as(ctypes.c_void_p),
                                      col.ctypes.data_as(ctypes.c_void_p),
                                      sh.ctypes.data_as(ctypes.c_void_p)) == 0
            assert (col == g.col).all() and (sh == g.shift).all()
            assert (np.bincount(row, minlength=g.M) == np.diff(g.row_ptr)).all()
            assert (np.diff(row) >= 0).all()
    # too small a buffer, a partial set of arrays, an unregistered graph
    small = ctypes.c_int(10)
    buf = np.zeros(10, np.int16)
    p = buf.ctypes.data_as(ctypes.c_void_p)
    assert lib.ldpc_get_graph(1, 384, None, None, ctypes.byref(small), p, p, p) == -1
    assert (buf == 0).all()
    assert lib.ldpc_get_graph(1, 384, None, None, ctypes.byref(small), p, None, None) == -1
    assert lib.ldpc_get_graph(2, 24, None, None, ctypes.byref(small), None, None, None) == -4
    assert lib.ldpc_graph_digest(1, 384, None) == -1


def test_library_graph_feeds_the_oracle(lib):
    # the helper the GPU comparisons use hands the oracle exactly the
    # registered table, sub-codes included
    from libgraph import library_graph
    from synth import make_graph
    for bg, Z, rows in ((1, 384, 46), (2, 16, 42), (1, 32, 7)):
        ref = make_graph(bg, Z, rows)
        got = library_graph(bg, Z, rows)
        assert (got.M, got.N, got.kb, got.n_punct) == (ref.M, ref.N, ref.kb, ref.n_punct)
        assert (got.row_ptr == ref.row_ptr).all()
        assert (got.col == ref.col).all() and (got.shift == ref.shift).all()


def test_tune_and_server_refusals_without_a_gpu(lib):
    # ldpc_tune only tunes int8 calls whose launch knobs are at their
    # defaults, and refuses the rest before any device work; the serving
    # queue is switched off and creates nothing
    from paper_2009_05534_amd import ldpc
    L = ldpc.lib()
    for field, value in (("precision", 1), ("lanes_per_row", 2), ("cw_per_block", 2),
                         ("msg_placement", 1), ("schedule", 1), ("max_workgroups", 4)):
        a = ldpc.Args()
        L.ldpc_args_init(ctypes.byref(a))
        a.bg, a.Z, a.rows, a.n_cw = 1, 384, 46, 4
        setattr(a, field, value)
        t = ldpc.Tuning()
        assert L.ldpc_tune(ctypes.byref(a), ctypes.byref(t)) == -1, field
    assert L.ldpc_tune(None, None) == -1
    h = ctypes.c_void_p()
    assert L.ldpc_server_create(64, 0, 10, 1, 0, ctypes.byref(h)) == -1
    assert not h.value
