"""Python binding of libldpc.so (include/ldpc.h): argument marshalling only.

Every step of decoding runs in the library's HIP kernels; torch supplies
device memory and the current stream. If the library is missing the binding
raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libldpc.so")

LDPC_I8 = 0
LDPC_F16 = 1
MSG_PLACEMENT = {"auto": 0, "lds": 1, "device": 2}
SCHEDULE = {"static": 0, "persistent": 1}
PAIRING = {"auto": 0, "codewords": 1, "rows": 2}
_ERRORS = {-1: "invalid argument", -2: "out of memory", -3: "HIP runtime error",
           -4: "no graph registered for (bg, Z)"}


class LdpcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_ERRORS.get(code, 'error')} ({code})")
        self.code = code


class Args(ctypes.Structure):
    _fields_ = [
        ("bg", ctypes.c_int), ("Z", ctypes.c_int), ("rows", ctypes.c_int), ("n_cw", ctypes.c_int),
        ("precision", ctypes.c_int), ("max_iter", ctypes.c_int), ("early_exit", ctypes.c_int),
        ("llr_in", ctypes.c_void_p),
        ("beta_q", ctypes.c_int), ("offset_q", ctypes.c_int), ("wq", ctypes.c_void_p),
        ("wq_iters", ctypes.c_int),
        ("beta_h", ctypes.c_uint16), ("offset_h", ctypes.c_uint16), ("wh", ctypes.c_void_p),
        ("wh_iters", ctypes.c_int),
        ("out_bits", ctypes.c_void_p), ("out_iters", ctypes.c_void_p),
        ("out_ok", ctypes.c_void_p), ("out_llr", ctypes.c_void_p),
        ("cw_per_block", ctypes.c_int), ("msg_placement", ctypes.c_int),
        ("lanes_per_row", ctypes.c_int), ("schedule", ctypes.c_int),
        ("max_workgroups", ctypes.c_int), ("pairing", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("lanes_per_row", ctypes.c_int), ("cw_per_block", ctypes.c_int),
                ("msg_placement", ctypes.c_int), ("schedule", ctypes.c_int),
                ("pairing", ctypes.c_int), ("ms", ctypes.c_float), ("candidates", ctypes.c_int)]


class Job(ctypes.Structure):
    _fields_ = [
        ("bg", ctypes.c_int), ("Z", ctypes.c_int), ("rows", ctypes.c_int), ("n_cw", ctypes.c_int),
        ("llr", ctypes.c_void_p), ("out_bits", ctypes.c_void_p), ("out_iters", ctypes.c_void_p),
        ("out_ok", ctypes.c_void_p), ("wq", ctypes.c_void_p), ("wq_iters", ctypes.c_int),
        ("split", ctypes.c_int),
    ]


PLAN_GRAPH = 1
PLAN_AUTOTUNE = 2

EXPORTS = ("ldpc_set_graph", "ldpc_query", "ldpc_get_graph", "ldpc_graph_digest", "ldpc_decode", "ldpc_args_init", "ldpc_decode_ex",
           "ldpc_decode_noalloc", "ldpc_tune",
           "ldpc_decode_batch", "ldpc_decode_batch_async", "ldpc_decode_batch_bytes", "ldpc_plan_create", "ldpc_plan_launch", "ldpc_plan_info",
           "ldpc_plan_destroy", "ldpc_nwms_loss_grad", "ldpc_server_create", "ldpc_server_submit",
           "ldpc_server_done", "ldpc_server_pump", "ldpc_server_destroy",
           "ldpc_strerror", "ldpc_last_hip_error",
           "ldpc_last_error_message", "ldpc_shutdown")

_lib = None


def lib():
    """Load libldpc.so (built in-tree by paper_2009_05534_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2009_05534_amd/build.py")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so the process runs one runtime whichever module is
        # imported first (two runtimes do not share the device).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, I = ctypes.c_void_p, ctypes.c_int
        L.ldpc_set_graph.argtypes = [I, I, I, I, P, P, P]
        L.ldpc_query.argtypes = [I, I, I, P, P, P, P]
        L.ldpc_decode.argtypes = [I, I, I, I, P, I, P, P, P]
        L.ldpc_get_graph.argtypes = [I, I, P, P, P, P, P, P]
        L.ldpc_graph_digest.argtypes = [I, I, P]
        L.ldpc_args_init.argtypes = [ctypes.POINTER(Args)]
        L.ldpc_args_init.restype = None
        L.ldpc_decode_ex.argtypes = [ctypes.POINTER(Args)]
        L.ldpc_decode_noalloc.argtypes = [ctypes.POINTER(Args)]
        L.ldpc_tune.argtypes = [ctypes.POINTER(Args), ctypes.POINTER(Tuning)]
        L.ldpc_decode_batch.argtypes = [ctypes.POINTER(Job), I, I, I, P]
        L.ldpc_decode_batch_async.argtypes = [ctypes.POINTER(Job), I, I, I, P,
                                              ctypes.POINTER(ctypes.c_size_t)]
        L.ldpc_decode_batch_bytes.argtypes = [ctypes.POINTER(Job), I,
                                              ctypes.POINTER(ctypes.c_size_t)]
        L.ldpc_plan_create.argtypes = [ctypes.POINTER(Job), I, I, I, I, P,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.ldpc_plan_launch.argtypes = [P, P]
        L.ldpc_plan_info.argtypes = [P, P, P, P]
        L.ldpc_plan_destroy.argtypes = [P]
        L.ldpc_plan_destroy.restype = None
        L.ldpc_nwms_loss_grad.argtypes = [I, I, I, I, P, P, I, P, P, ctypes.c_float, P, P, P, P]
        L.ldpc_server_create.argtypes = [I, I, I, I, I, ctypes.POINTER(ctypes.c_void_p)]
        L.ldpc_server_submit.argtypes = [P, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint),
                                         ctypes.POINTER(ctypes.c_int)]
        L.ldpc_server_done.argtypes = [P, ctypes.c_uint]
        L.ldpc_server_pump.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.ldpc_server_destroy.argtypes = [P]
        L.ldpc_strerror.argtypes = [I]
        L.ldpc_strerror.restype = ctypes.c_char_p
        L.ldpc_last_hip_error.argtypes = []
        L.ldpc_last_error_message.argtypes = []
        L.ldpc_last_error_message.restype = ctypes.c_char_p
        L.ldpc_shutdown.argtypes = []
        L.ldpc_shutdown.restype = None
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        detail = lib().ldpc_last_error_message().decode()
        raise LdpcError(rc, what + (f" [{detail}]" if detail else ""))


def set_graph(bg: int, Z: int, m_rows: int, kb: int, row_ptr, col, shift) -> None:
    """Register base graph ``bg`` lifted by ``Z`` (host arrays, copied)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int16)
    s = np.ascontiguousarray(shift, dtype=np.int16)
    _check(lib().ldpc_set_graph(bg, Z, m_rows, kb, rp.ctypes.data, c.ctypes.data, s.ctypes.data),
           "ldpc_set_graph")


def register(g) -> None:
    """Register a full graph object with fields bg, Z, M, kb, row_ptr, col, shift."""
    set_graph(g.bg, g.Z, g.M, g.kb, g.row_ptr, g.col, g.shift)


def query(bg: int, Z: int, rows: int) -> tuple[int, int, int, int]:
    """(K, T, Nc, E) of the sub-code keeping ``rows`` block rows."""
    out = [ctypes.c_int() for _ in range(4)]
    _check(lib().ldpc_query(bg, Z, rows, *[ctypes.addressof(o) for o in out]), "ldpc_query")
    return tuple(o.value for o in out)


def get_graph(bg: int, Z: int):
    """The registered graph (bg, Z) as (m_rows, kb, row, col, shift): one
    entry per nonzero block, row-major, columns ascending (numpy int16)."""
    L = lib()
    m, kb, nnz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(L.ldpc_get_graph(bg, Z, ctypes.byref(m), ctypes.byref(kb), ctypes.byref(nnz),
                            None, None, None), "ldpc_get_graph")
    row, col, shift = (np.empty(nnz.value, np.int16) for _ in range(3))
    _check(L.ldpc_get_graph(bg, Z, ctypes.byref(m), ctypes.byref(kb), ctypes.byref(nnz),
                            row.ctypes.data, col.ctypes.data, shift.ctypes.data),
           "ldpc_get_graph")
    return m.value, kb.value, row, col, shift


def graph_digest(bg: int, Z: int) -> int:
    """64-bit FNV-1a digest of the registered graph (see include/ldpc.h)."""
    out = ctypes.c_uint64()
    _check(lib().ldpc_graph_digest(bg, Z, ctypes.byref(out)), "ldpc_graph_digest")
    return out.value


def _require(t, shape, itemsize, name):
    """Device tensor of exactly ``shape``, contiguous, with ``itemsize``-byte
    elements: the library trusts the sizes it is given."""
    if (not t.is_cuda or tuple(t.shape) != tuple(shape) or not t.is_contiguous()
            or t.element_size() != itemsize):
        raise ValueError(f"{name}: need a contiguous device tensor {tuple(shape)} "
                         f"of {itemsize}-byte elements, got {tuple(t.shape)} {t.dtype}")


def _f16_bits(v: float) -> int:
    return int(np.array([v], dtype=np.float16).view(np.uint16)[0])


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def decode_into(llr, bg: int, Z: int, rows: int, out_bits, out_iters, *, max_iter: int = 10,
                precision: str = "i8", early_exit: bool = True, beta: float | None = None,
                offset: float = 0, weights=None, out_ok=None, out_llr=None,
                cw_per_block: int = 0, msg_placement: str = "auto", stream=None,
                noalloc: bool = False, lanes_per_row: int = 0, tune: bool = False,
                schedule: str = "static", max_workgroups: int = 0, pairing: str = "auto"):
    """Decode int8 LLRs [n_cw, T] (device tensor) into preallocated outputs.

    ``pairing`` (int8): "codewords" (two codewords per lane), "rows" (check
    rows u and u + Z/2 of one codeword per lane) or "auto" (rows for small
    batches of lifts above 256).

    ``noalloc``: call ldpc_decode_noalloc (messages in the library's static
    per-device scratch; nothing is allocated) instead of ldpc_decode_ex.
    ``tune``: call ldpc_tune instead (times the launch configurations, keeps
    the fastest for this shape and batch size, writes the outputs) and
    return the choice as a dict.

    ``weights``: per-(iteration, row) normalisation, a device tensor uint8
    [iters, rows] (Q1.7, i8) or float16 [iters, rows] (f16).
    ``beta``/``offset``: plain normalisation (i8: beta in units of 1/128 is
    taken from ``round(128*beta)``, offset an integer; f16: binary16 values).
    """
    n_cw = int(llr.shape[0])
    K, T, Nc, _ = query(bg, Z, rows)
    _require(llr, (n_cw, T), 1, "llr")
    _require(out_bits, (n_cw, K // 8), 1, "out_bits")
    _require(out_iters, (n_cw,), 4, "out_iters")
    if out_ok is not None:
        _require(out_ok, (n_cw,), 1, "out_ok")
    if out_llr is not None:
        _require(out_llr, (n_cw, Nc), 1 if precision == "i8" else 2, "out_llr")
    if weights is not None:
        if weights.dim() != 2 or weights.shape[1] != rows or weights.shape[0] < 1:
            raise ValueError("weights must be [iters, rows]")
        _require(weights, tuple(weights.shape), 1 if precision == "i8" else 2, "weights")
    a = Args()
    lib().ldpc_args_init(ctypes.byref(a))
    a.bg, a.Z, a.rows, a.n_cw = bg, Z, rows, n_cw
    a.precision = LDPC_I8 if precision == "i8" else LDPC_F16
    if precision not in ("i8", "f16"):
        raise ValueError("precision must be 'i8' or 'f16'")
    a.max_iter = max_iter
    a.early_exit = 1 if early_exit else 0
    a.llr_in = llr.data_ptr()
    if precision == "i8":
        if beta is not None:
            a.beta_q = int(round(beta * 128))
        a.offset_q = int(offset)
        if weights is not None:
            a.wq = weights.data_ptr()
            a.wq_iters = int(weights.shape[0])
    else:
        if beta is not None:
            a.beta_h = _f16_bits(beta)
        a.offset_h = _f16_bits(offset)
        if weights is not None:
            a.wh = weights.data_ptr()
            a.wh_iters = int(weights.shape[0])
    a.out_bits = out_bits.data_ptr()
    a.out_iters = out_iters.data_ptr()
    a.out_ok = out_ok.data_ptr() if out_ok is not None else None
    a.out_llr = out_llr.data_ptr() if out_llr is not None else None
    a.cw_per_block = cw_per_block
    a.msg_placement = MSG_PLACEMENT[msg_placement]
    a.lanes_per_row = lanes_per_row
    if schedule not in SCHEDULE:
        raise ValueError("schedule must be 'static' or 'persistent'")
    a.schedule = SCHEDULE[schedule]
    a.max_workgroups = max_workgroups
    if pairing not in PAIRING:
        raise ValueError("pairing must be 'auto', 'codewords' or 'rows'")
    a.pairing = PAIRING[pairing]
    a.stream = _stream_ptr(stream)
    if tune:
        t = Tuning()
        _check(lib().ldpc_tune(ctypes.byref(a), ctypes.byref(t)), "ldpc_tune")
        return {"lanes_per_row": t.lanes_per_row, "cw_per_block": t.cw_per_block,
                "msg_placement": {v: k for k, v in MSG_PLACEMENT.items()}[t.msg_placement],
                "schedule": "persistent" if t.schedule == 1 else "static",
                "pairing": {v: k for k, v in PAIRING.items()}[t.pairing],
                "ms": t.ms, "candidates": t.candidates}
    if noalloc:
        _check(lib().ldpc_decode_noalloc(ctypes.byref(a)), "ldpc_decode_noalloc")
    else:
        _check(lib().ldpc_decode_ex(ctypes.byref(a)), "ldpc_decode_ex")


def decode(llr, bg: int, Z: int, rows: int, *, max_iter: int = 10, precision: str = "i8",
           early_exit: bool = True, beta: float | None = None, offset: float = 0, weights=None,
           want_ok: bool = True, want_llr: bool = False, cw_per_block: int = 0,
           msg_placement: str = "auto", stream=None, noalloc: bool = False,
           lanes_per_row: int = 0, schedule: str = "static", max_workgroups: int = 0,
           pairing: str = "auto"):
    """Allocate outputs with torch on llr's device and decode (through
    ldpc_decode_noalloc when ``noalloc``; the outputs are still allocated
    here, by torch).

    Returns (bits uint8 [n, K/8], iters int32 [n], ok bool [n] or None,
    llr int8/float16 [n, Nc] or None)."""
    import torch
    K, T, Nc, E = query(bg, Z, rows)
    if llr.dim() != 2 or llr.dtype != torch.int8:
        raise ValueError(f"llr must be a device int8 tensor [n_cw, {T}]")
    n = int(llr.shape[0])
    dev = llr.device
    bits = torch.empty((n, K // 8), dtype=torch.uint8, device=dev)
    iters = torch.empty(n, dtype=torch.int32, device=dev)
    ok = torch.empty(n, dtype=torch.uint8, device=dev) if want_ok else None
    out = None
    if want_llr:
        out = torch.empty((n, Nc), dtype=torch.int8 if precision == "i8" else torch.float16,
                          device=dev)
    decode_into(llr, bg, Z, rows, bits, iters, max_iter=max_iter, precision=precision,
                early_exit=early_exit, beta=beta, offset=offset, weights=weights, out_ok=ok,
                out_llr=out, cw_per_block=cw_per_block, msg_placement=msg_placement,
                stream=stream, noalloc=noalloc, lanes_per_row=lanes_per_row,
                schedule=schedule, max_workgroups=max_workgroups, pairing=pairing)
    return bits, iters, (ok.bool() if ok is not None else None), out


def nwms_loss_grad(llr, cbits, w, bg: int, Z: int, rows: int, *, scale: float = 4.0,
                   iter_w=None, want_llr: bool = False, stream=None):
    """Learned weighted min-sum on the GPU: fp32 unrolled forward pass over
    w.shape[0] iterations, loss per codeword and the gradient of the summed
    loss with respect to w [n_iter, rows] (hand-written backward kernel).

    llr float32 [n, T] and cbits uint8 [n, Nc] are device tensors; iter_w a
    float32 device tensor [n_iter] of per-iteration loss weights or None
    (1/n_iter each); returns (loss [n], grad [n_iter, rows], final
    posteriors [n, Nc] or None)."""
    import torch
    K, T, Nc, E = query(bg, Z, rows)
    n = int(llr.shape[0])
    _require(llr, (n, T), 4, "llr")
    _require(cbits, (n, Nc), 1, "cbits")
    if w.dim() != 2 or w.shape[1] != rows:
        raise ValueError("w must be [n_iter, rows]")
    _require(w, tuple(w.shape), 4, "w")
    if iter_w is not None:
        _require(iter_w, (int(w.shape[0]),), 4, "iter_w")
    dev = llr.device
    loss = torch.empty(n, dtype=torch.float32, device=dev)
    grad = torch.empty(tuple(w.shape), dtype=torch.float32, device=dev)
    out = torch.empty((n, Nc), dtype=torch.float32, device=dev) if want_llr else None
    _check(lib().ldpc_nwms_loss_grad(bg, Z, rows, n, llr.data_ptr(), cbits.data_ptr(),
                                     int(w.shape[0]), w.data_ptr(),
                                     iter_w.data_ptr() if iter_w is not None else None,
                                     float(scale), loss.data_ptr(),
                                     grad.data_ptr(), out.data_ptr() if out is not None else None,
                                     _stream_ptr(stream)), "ldpc_nwms_loss_grad")
    return loss, grad, out


class BatchJob:
    """One job of a mixed-shape batch: codewords of one shape with their
    device buffers (outputs allocated here unless given)."""

    def __init__(self, llr, bg: int, Z: int, rows: int, weights=None, out_bits=None,
                 out_iters=None, out_ok=None, split: bool = False):
        import torch
        K, T, Nc, E = query(bg, Z, rows)
        n = int(llr.shape[0])
        _require(llr, (n, T), 1, "llr")
        dev = llr.device
        self.bg, self.Z, self.rows, self.n = bg, Z, rows, n
        self.split = bool(split)  # small tasks (one pair / one codeword as row pairs)
        self.llr = llr
        self.out_bits = out_bits if out_bits is not None else torch.empty(
            (n, K // 8), dtype=torch.uint8, device=dev)
        self.out_iters = out_iters if out_iters is not None else torch.empty(
            n, dtype=torch.int32, device=dev)
        self.out_ok = out_ok if out_ok is not None else torch.empty(n, dtype=torch.uint8,
                                                                    device=dev)
        _require(self.out_bits, (n, K // 8), 1, "out_bits")
        _require(self.out_iters, (n,), 4, "out_iters")
        _require(self.out_ok, (n,), 1, "out_ok")
        self.weights = weights
        if weights is not None:
            if weights.dim() != 2 or weights.shape[1] != rows:
                raise ValueError("weights must be [iters, rows]")
            _require(weights, tuple(weights.shape), 1, "weights")

    def c_struct(self) -> Job:
        return Job(self.bg, self.Z, self.rows, self.n, self.llr.data_ptr(),
                   self.out_bits.data_ptr(), self.out_iters.data_ptr(), self.out_ok.data_ptr(),
                   self.weights.data_ptr() if self.weights is not None else None,
                   int(self.weights.shape[0]) if self.weights is not None else 0,
                   int(self.split))


def _job_array(jobs):
    """ctypes array of Job structs from BatchJob objects or Job structs."""
    arr = (Job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j if isinstance(j, Job) else j.c_struct()
    return arr


def decode_batch(jobs, *, max_iter: int = 10, early_exit: bool = True, stream=None) -> None:
    """One persistent launch over all jobs; waits for the stream."""
    arr = _job_array(jobs)
    _check(lib().ldpc_decode_batch(arr, len(jobs), max_iter, int(early_exit), _stream_ptr(stream)),
           "ldpc_decode_batch")


def decode_batch_async(jobs, *, max_iter: int = 10, early_exit: bool = True,
                       stream=None) -> int:
    """One persistent launch over all jobs, enqueued on `stream` without
    waiting; returns the device bytes the launch holds until it completes.
    The caller keeps the jobs' tensors alive until then."""
    arr = _job_array(jobs)
    nb = ctypes.c_size_t()
    _check(lib().ldpc_decode_batch_async(arr, len(jobs), max_iter, int(early_exit),
                                         _stream_ptr(stream), ctypes.byref(nb)),
           "ldpc_decode_batch_async")
    return int(nb.value)


def decode_batch_bytes(jobs) -> int:
    """Device bytes decode_batch_async would hold in flight for these jobs
    (computed without allocating or launching). ``jobs``: BatchJob objects
    or their Job structs (whose buffers the caller keeps alive)."""
    arr = _job_array(jobs)
    nb = ctypes.c_size_t()
    _check(lib().ldpc_decode_batch_bytes(arr, len(jobs), ctypes.byref(nb)),
           "ldpc_decode_batch_bytes")
    return int(nb.value)


class Plan:
    """Reusable mixed-shape plan bound to the jobs' buffers; optionally a HIP
    graph and autotuned grid (see include/ldpc.h)."""

    def __init__(self, jobs, *, max_iter: int = 10, early_exit: bool = True, graph: bool = False,
                 autotune: bool = False, stream=None):
        self.jobs = list(jobs)  # keeps the tensors alive
        arr = _job_array(self.jobs)
        h = ctypes.c_void_p()
        flags = (PLAN_GRAPH if graph else 0) | (PLAN_AUTOTUNE if autotune else 0)
        _check(lib().ldpc_plan_create(arr, len(self.jobs), max_iter, int(early_exit), flags,
                                      _stream_ptr(stream), ctypes.byref(h)), "ldpc_plan_create")
        self._h = h

    def launch(self, stream=None) -> None:
        _check(lib().ldpc_plan_launch(self._h, _stream_ptr(stream)), "ldpc_plan_launch")

    def info(self) -> dict:
        g, n, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
        _check(lib().ldpc_plan_info(self._h, ctypes.byref(g), ctypes.byref(n), ctypes.byref(t)),
               "ldpc_plan_info")
        return {"grid": g.value, "n_tasks": n.value, "tuned_ms": t.value}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().ldpc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def job_record(llr, bg: int, Z: int, rows: int, out_bits, out_iters, out_ok=None,
               weights=None) -> Job:
    """The C job record of one serving job: llr a device int8 tensor
    [n, T]; outputs device tensors or pinned host tensors (the serving
    kernel writes pinned ones directly); weights a device uint8 tensor
    [iters, rows] or None. The caller keeps every tensor alive until the
    job's tasks are done."""
    K, T, Nc, E = query(bg, Z, rows)
    n = int(llr.shape[0])
    _require(llr, (n, T), 1, "llr")
    for t, shape, size, name in ((out_bits, (n, K // 8), 1, "out_bits"),
                                 (out_iters, (n,), 4, "out_iters"),
                                 (out_ok, (n,), 1, "out_ok")):
        if t is None:
            if name != "out_ok":
                raise ValueError(f"{name} is required")
            continue
        if not (t.is_cuda or t.is_pinned()) or tuple(t.shape) != shape or \
                not t.is_contiguous() or t.element_size() != size:
            raise ValueError(f"{name}: need a contiguous device or pinned tensor {shape}")
    if weights is not None:
        if weights.dim() != 2 or weights.shape[1] != rows:
            raise ValueError("weights must be [iters, rows]")
        _require(weights, tuple(weights.shape), 1, "weights")
    return Job(bg, Z, rows, n, llr.data_ptr(), out_bits.data_ptr(), out_iters.data_ptr(),
               out_ok.data_ptr() if out_ok is not None else None,
               weights.data_ptr() if weights is not None else None,
               int(weights.shape[0]) if weights is not None else 0)


class QueueServer:
    """The library's serving queue (ldpc_server_*): a persistent decode
    kernel fed from a ring of task descriptors in pinned host memory."""

    def __init__(self, capacity: int = 4096, grid: int = 0, max_iter: int = 10,
                 early_exit: bool = True, idle_polls: int = 0):
        h = ctypes.c_void_p()
        _check(lib().ldpc_server_create(capacity, grid, max_iter, int(early_exit), idle_polls,
                                        ctypes.byref(h)), "ldpc_server_create")
        self._h = h

    def submit(self, job: Job) -> tuple[int, int]:
        """Appends the job's tasks; returns (first ticket, number of tasks),
        or None when the ring has no room (nothing appended)."""
        first, n = ctypes.c_uint(), ctypes.c_int()
        rc = lib().ldpc_server_submit(self._h, ctypes.byref(job), ctypes.byref(first),
                                      ctypes.byref(n))
        if rc == -2:
            return None
        _check(rc, "ldpc_server_submit")
        return first.value, n.value

    def done(self, ticket: int) -> bool:
        return lib().ldpc_server_done(self._h, ticket) == 1

    def pump(self) -> tuple[int, int]:
        """Relaunches the kernel if tasks are pending and it has left;
        returns (tasks outstanding, kernel launches so far)."""
        o, n = ctypes.c_int(), ctypes.c_int()
        _check(lib().ldpc_server_pump(self._h, ctypes.byref(o), ctypes.byref(n)),
               "ldpc_server_pump")
        return o.value, n.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(lib().ldpc_server_destroy(self._h), "ldpc_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
