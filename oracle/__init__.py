"""CPU oracle for layered normalised min-sum LDPC decoding -- TEST
INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg may import this package. The decoder product never calls it,
and it shares no code with the GPU path (the graph arrives as plain arrays).

``ldpc_oracle.c`` holds the decoding arithmetic (int8 saturating, binary16
emulated, double); this module only marshals numpy arrays through ctypes.
``bruteforce.py`` holds exhaustive-search references for tiny codes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldpc_oracle.c")
_LIB = os.path.join(_HERE, "libldpc_oracle.so")
_lib = None


def _compile(out: str, extra: list[str]) -> None:
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O3", *extra, "-std=c11", "-Wall", "-Wextra", "-fPIC",
                           "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O3 (plain C, no intrinsics; generic x86-64
    code, so the built library runs on any host it is copied to)."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, [])
    return _LIB


def use_native_build(directory: str) -> str:
    """Compile the oracle with -O3 -march=native for the host it runs on into
    ``directory`` and make this module use that build (the CPU baseline's
    timing; the arithmetic is the same C source). Returns the library path."""
    global _lib
    path = os.path.join(directory, "libldpc_oracle_native.so")
    _compile(path, ["-march=native"])
    _lib = None
    _load(path)
    return path


def _load(path: str | None = None):
    global _lib
    if _lib is None:
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        lib.oracle_decode_i8.argtypes = [I, I, I, I, I, P, P, P, I, P, I, I, I, P, I, P, P, P, P, I]
        lib.oracle_decode_f16.argtypes = [I, I, I, I, I, P, P, P, I, P, I, I, ctypes.c_uint16,
                                          ctypes.c_uint16, P, I, P, P, P, P, I]
        lib.oracle_decode_f64.argtypes = [I, I, I, I, I, P, P, P, I, P, I, I, ctypes.c_double,
                                          ctypes.c_double, P, I, P, P, P, P, I]
        lib.oracle_decode_bp_f64.argtypes = [I, I, I, I, I, P, P, P, I, P, I, I, I, I,
                                             ctypes.c_double, P, P, P, P, I]
        lib.oracle_decode_bp_f64.restype = ctypes.c_int
        lib.oracle_nwms_grad_f64.argtypes = [I, I, I, I, P, P, P, I, P, P, I, P, P,
                                             ctypes.c_double, P, P]
        lib.oracle_nwms_grad_f64.restype = ctypes.c_int
        lib.oracle_f64_to_f16.argtypes = [P, P, ctypes.c_long]
        lib.oracle_f16_to_f64.argtypes = [P, P, ctypes.c_long]
        for f in (lib.oracle_decode_i8, lib.oracle_decode_f16, lib.oracle_decode_f64):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_args(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int16)
    sh = np.ascontiguousarray(g.shift, dtype=np.int16)
    return (g.M, g.N, g.Z, g.n_punct, g.K), (rp, col, sh)


def f64_to_f16(v) -> np.ndarray:
    """Round doubles to IEEE binary16 bit patterns (nearest, ties to even)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(v.shape, dtype=np.uint16)
    _load().oracle_f64_to_f16(_ptr(v), _ptr(out), v.size)
    return out


def f16_to_f64(h) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint16)
    out = np.empty(h.shape, dtype=np.float64)
    _load().oracle_f16_to_f64(_ptr(h), _ptr(out), h.size)
    return out


def _outputs(g, n_cw, want_llr, llr_dtype):
    return (np.zeros((n_cw, (g.K + 7) // 8), np.uint8), np.zeros(n_cw, np.int32),
            np.zeros(n_cw, np.uint8),
            np.zeros((n_cw, g.N * g.Z), llr_dtype) if want_llr else None)


def decode_i8(g, q, max_iter=10, early_exit=True, delta=0, wq=None, want_llr=False,
              n_threads=1):
    """int8 saturating layered min-sum. q int8 [n_cw, T]; wq uint8 [iters, M]
    Q1.7 multipliers (None: 96, i.e. beta = 3/4). Returns (bits, iters, ok, llr)."""
    q = np.ascontiguousarray(q, dtype=np.int8)
    n_cw = q.shape[0]
    assert q.shape == (n_cw, g.T)
    dims, (rp, col, sh) = _graph_args(g)
    wq_a = None if wq is None else np.ascontiguousarray(wq, dtype=np.uint8)
    if wq_a is not None:
        assert wq_a.ndim == 2 and wq_a.shape[1] == g.M
    bits, iters, ok, llr = _outputs(g, n_cw, want_llr, np.int8)
    rc = _load().oracle_decode_i8(*dims, _ptr(rp), _ptr(col), _ptr(sh), n_cw, _ptr(q), max_iter,
                                  int(early_exit), int(delta), _ptr(wq_a),
                                  0 if wq_a is None else wq_a.shape[0], _ptr(bits), _ptr(iters),
                                  _ptr(ok), _ptr(llr), n_threads)
    if rc != 0:
        raise ValueError(f"oracle_decode_i8 failed ({rc})")
    return bits, iters, ok.astype(bool), llr


def decode_f16(g, q, max_iter=10, early_exit=True, beta=0.75, delta=0.0, wh=None,
               want_llr=False, n_threads=1):
    """binary16-emulated layered min-sum. Returns (bits, iters, ok, llr_f16_bits)."""
    q = np.ascontiguousarray(q, dtype=np.int8)
    n_cw = q.shape[0]
    assert q.shape == (n_cw, g.T)
    dims, (rp, col, sh) = _graph_args(g)
    wh_a = None if wh is None else np.ascontiguousarray(wh, dtype=np.uint16)
    bits, iters, ok, llr = _outputs(g, n_cw, want_llr, np.uint16)
    b16 = int(f64_to_f16(np.array([beta]))[0])
    d16 = int(f64_to_f16(np.array([delta]))[0])
    rc = _load().oracle_decode_f16(*dims, _ptr(rp), _ptr(col), _ptr(sh), n_cw, _ptr(q), max_iter,
                                   int(early_exit), b16, d16, _ptr(wh_a),
                                   0 if wh_a is None else wh_a.shape[0], _ptr(bits), _ptr(iters),
                                   _ptr(ok), _ptr(llr), n_threads)
    if rc != 0:
        raise ValueError(f"oracle_decode_f16 failed ({rc})")
    return bits, iters, ok.astype(bool), llr


def decode_f64(g, llr, max_iter=10, early_exit=True, beta=0.75, delta=0.0, w=None,
               want_llr=False, n_threads=1):
    """Double-precision layered min-sum on real-valued LLRs [n_cw, T]."""
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    n_cw = llr.shape[0]
    assert llr.shape == (n_cw, g.T)
    dims, (rp, col, sh) = _graph_args(g)
    w_a = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    bits, iters, ok, out = _outputs(g, n_cw, want_llr, np.float64)
    rc = _load().oracle_decode_f64(*dims, _ptr(rp), _ptr(col), _ptr(sh), n_cw, _ptr(llr),
                                   max_iter, int(early_exit), float(beta), float(delta), _ptr(w_a),
                                   0 if w_a is None else w_a.shape[0], _ptr(bits), _ptr(iters),
                                   _ptr(ok), _ptr(out), n_threads)
    if rc != 0:
        raise ValueError(f"oracle_decode_f64 failed ({rc})")
    return bits, iters, ok.astype(bool), out


def decode_bp(g, llr, rule="spa", schedule="layered", max_iter=10, early_exit=True,
              beta=0.75, want_llr=False, n_threads=1):
    """Double-precision belief propagation on real-valued LLRs [n_cw, T] with
    the sum-product ("spa") or normalised min-sum ("minsum", beta) check rule
    on the layered or flooding schedule (context for the decoder's choices)."""
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    n_cw = llr.shape[0]
    assert llr.shape == (n_cw, g.T)
    rules = {"minsum": 0, "spa": 1}
    schedules = {"layered": 0, "flooding": 1}
    dims, (rp, col, sh) = _graph_args(g)
    bits, iters, ok, out = _outputs(g, n_cw, want_llr, np.float64)
    rc = _load().oracle_decode_bp_f64(*dims, _ptr(rp), _ptr(col), _ptr(sh), n_cw, _ptr(llr),
                                      max_iter, int(early_exit), rules[rule],
                                      schedules[schedule], float(beta), _ptr(bits), _ptr(iters),
                                      _ptr(ok), _ptr(out), n_threads)
    if rc != 0:
        raise ValueError(f"oracle_decode_bp_f64 failed ({rc})")
    return bits, iters, ok.astype(bool), out


def nwms_loss_grad(g, llr, cbits, w, scale=4.0, iter_w=None):
    """Learned weighted min-sum in double precision: per-codeword loss
    (over iterations t weighted by iter_w[t], default 1/n_iter each, the
    mean over bits of the BCE of sigmoid(-L/scale) against the codeword)
    and the exact gradient of the summed loss with respect to the weights
    w [n_iter, M]. llr [n_cw, T] real, cbits [n_cw, N*Z] 0/1."""
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    cb = np.ascontiguousarray(cbits, dtype=np.uint8)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n_cw = llr.shape[0]
    assert llr.shape == (n_cw, g.T) and cb.shape == (n_cw, g.N * g.Z)
    assert w.ndim == 2 and w.shape[1] == g.M
    dims, (rp, col, sh) = _graph_args(g)
    loss = np.zeros(n_cw)
    grad = np.zeros_like(w)
    lam = None
    if iter_w is not None:
        lam = np.ascontiguousarray(iter_w, dtype=np.float64)
        assert lam.shape == (w.shape[0],)
    rc = _load().oracle_nwms_grad_f64(g.M, g.N, g.Z, g.n_punct, _ptr(rp), _ptr(col), _ptr(sh),
                                      n_cw, _ptr(llr), _ptr(cb), w.shape[0], _ptr(w),
                                      _ptr(lam) if lam is not None else None,
                                      float(scale), _ptr(loss), _ptr(grad))
    if rc != 0:
        raise ValueError(f"oracle_nwms_grad_f64 failed ({rc})")
    return loss, grad


def unpack_bits(bits: np.ndarray, K: int) -> np.ndarray:
    """Packed LSB-first bytes [n, ceil(K/8)] -> 0/1 uint8 [n, K]."""
    return np.unpackbits(bits, axis=1, bitorder="little")[:, :K]
