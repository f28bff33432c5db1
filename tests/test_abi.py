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
    a.bg = 7
    assert lib_.ldpc_decode_ex(ctypes.byref(a)) == -4
    assert lib_.ldpc_strerror(-4) == b"no graph registered for (bg, Z)"
