"""Thin ctypes binding of libnf.so (include/nf.h), names as in the C ABI.

Marshalling only: every step of a fold runs in the library's HIP kernels.
PyTorch supplies device memory and streams: once the library is loaded, its
device buffers come from torch's caching allocator through the library's
allocator hook (``nf_set_allocator``; set NF_TORCH_ALLOCATOR=0 to keep
hipMalloc), and the ``*_dev`` variants run on torch streams.
The binding raises ``NFError`` for every negative return code and fails loudly
when the library is missing: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnf.so")

NF_OK = 0
NF_E_INVAL = -1
NF_E_NOMEM = -2
NF_E_DEVICE = -3
NF_E_BUSY = -4
NF_E_NOTFOUND = -5
NF_E_TOOLONG = -6
NF_E_TIMEOUT = -7
NF_E_ABORTED = -8
NF_MAX_N = 65534
NF_WANT_TABLE = 1
NF_WANT_STRUCTURE = 2

_CODE_NAMES = {
    NF_E_INVAL: "NF_E_INVAL", NF_E_NOMEM: "NF_E_NOMEM", NF_E_DEVICE: "NF_E_DEVICE",
    NF_E_BUSY: "NF_E_BUSY", NF_E_NOTFOUND: "NF_E_NOTFOUND", NF_E_TOOLONG: "NF_E_TOOLONG",
    NF_E_TIMEOUT: "NF_E_TIMEOUT", NF_E_ABORTED: "NF_E_ABORTED",
}

# every symbol include/nf.h declares
EXPORTS = [
    "nf_last_error", "nf_init", "nf_shutdown", "nf_set_allocator", "nf_encode",
    "nf_precompute_R", "nf_copy_R", "nf_fold", "nf_fold_structure",
    "nf_fold_dev", "nf_fold_dev_noalloc", "nf_batch_create", "nf_batch_run", "nf_batch_scores", "nf_batch_table",
    "nf_batch_info", "nf_batch_structures", "nf_batch_destroy", "nf_fold_batch", "nf_serve_config", "nf_fold_bytes",
    "nf_submit", "nf_poll", "nf_wait", "nf_poll_ex", "nf_serve_stats", "nf_autotune_q",
    "nf_autotune_target", "nf_autotune_wide", "nf_autotune", "nf_profile_fold", "nf_lds_gather_rate",
]


class NFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_CODE_NAMES.get(code, "NF_E_?"), code, msg))
        self.code = code


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("active", ctypes.c_int64),
                ("pending", ctypes.c_int64), ("budget_bytes", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t), ("steps_fused", ctypes.c_int64)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4),
                ("lookups", ctypes.c_double * 4), ("splits", ctypes.c_double * 4), ("cells", ctypes.c_double * 4),
                ("q", ctypes.c_int), ("tile", ctypes.c_int), ("tiles_per_side", ctypes.c_int),
                ("stages", ctypes.c_int), ("wide", ctypes.c_int)]


KERNEL_NAMES = ("k_diag", "k_tile", "k_between", "k_stage")

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libnf.so (built by ``paper_1307_7820_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libnf.so not found at %s; build it with "
                          "`python -m paper_1307_7820_amd.build`" % path)
    # PyTorch ships its own HIP runtime (SONAME libamdhip64.so.7).  Importing
    # torch first makes libnf.so bind to that same runtime instance, so torch's
    # streams and device pointers are valid in the library and only one
    # runtime owns the device.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    c_int, c_i64, c_sz, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
    sig = {
        "nf_last_error": (ctypes.c_char_p, []),
        "nf_init": (c_int, [c_int]),
        "nf_shutdown": (None, []),
        "nf_set_allocator": (c_int, [vp, vp, vp]),
        "nf_encode": (c_int, [ctypes.c_char_p, c_int, vp]),
        "nf_precompute_R": (c_int, [c_int]),
        "nf_copy_R": (c_int, [c_int, vp, c_sz]),
        "nf_fold": (c_int, [ctypes.c_char_p, c_int, c_int, vp]),
        "nf_fold_structure": (c_int, [ctypes.c_char_p, c_int, c_int, vp]),
        "nf_fold_dev": (c_int, [vp, c_int, c_int, vp, vp, vp]),
        "nf_fold_dev_noalloc": (c_int, [vp, c_int, c_int, vp, vp, vp]),
        "nf_batch_create": (c_int, [vp, vp, c_int, c_int, ctypes.POINTER(vp)]),
        "nf_batch_run": (c_int, [vp, vp]),
        "nf_batch_scores": (c_int, [vp, vp]),
        "nf_batch_table": (c_int, [vp, c_int, vp]),
        "nf_batch_structures": (c_int, [vp, vp]),
        "nf_batch_info": (c_int, [vp, ctypes.POINTER(c_int), ctypes.POINTER(c_sz)]),
        "nf_batch_destroy": (None, [vp]),
        "nf_fold_batch": (c_int, [vp, vp, c_int, c_int, vp, vp]),
        "nf_serve_config": (c_int, [c_sz, c_int, c_int]),
        "nf_fold_bytes": (c_sz, [c_int, c_int]),
        "nf_submit": (c_i64, [ctypes.c_char_p, c_int, c_int, c_int]),
        "nf_poll": (c_int, [c_i64, vp, vp]),
        "nf_wait": (c_int, [c_i64, c_int, vp, vp]),
        "nf_poll_ex": (c_int, [c_i64, c_int, vp, vp, vp]),
        "nf_serve_stats": (c_int, [ctypes.POINTER(ServeStats)]),
        "nf_autotune_q": (c_int, [c_int]),
        "nf_autotune_target": (c_int, [c_int, c_int]),
        "nf_autotune_wide": (c_int, [c_int, c_int]),
        "nf_autotune": (c_int, [c_int, c_int, c_int, c_int]),
        "nf_profile_fold": (c_int, [vp, c_int, c_int, c_int, vp, ctypes.POINTER(KernelProfile)]),
        "nf_lds_gather_rate": (c_int, [c_int, c_int, ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    if os.environ.get("NF_TORCH_ALLOCATOR", "1") != "0":
        use_torch_allocator()
    return L


# ---------------------------------------------------------------- device memory

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
# Every hook ever installed stays referenced: a buffer goes back through the
# hook it came from, which may be an earlier one.
_hooks: list = []
_live_batches = None  # weakref.WeakSet of Batch objects, closed at exit
_exit_registered = False


def nf_set_allocator(alloc=None, free=None) -> None:
    """Install a device memory hook: ``alloc(nbytes) -> address`` (0 on
    failure) and ``free(address)``; both None restores hipMalloc/hipFree."""
    L = load()
    if alloc is None and free is None:
        _check(L.nf_set_allocator(None, None, None))
        return
    if alloc is None or free is None:
        raise ValueError("nf_set_allocator needs both functions, or neither")

    def a(nbytes, ctx):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:
            return None  # the library reports NF_E_NOMEM

    def f(ptr, ctx):
        free(int(ptr))

    fa, ff = _ALLOC_FN(a), _FREE_FN(f)
    _hooks.append((fa, ff))
    _check(L.nf_set_allocator(ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ff, ctypes.c_void_p), None))
    _register_exit()


def use_torch_allocator() -> None:
    """Let torch's caching allocator supply every device buffer of the
    library (on the library's device and the calling thread's current torch
    stream; the library waits for the device before it hands a block back)."""
    import torch

    def alloc(nbytes):
        return torch.cuda.caching_allocator_alloc(nbytes)

    def free(ptr):
        torch.cuda.caching_allocator_delete(ptr)

    nf_set_allocator(alloc, free)


def _register_exit() -> None:
    """Release the library's buffers while the interpreter (and the hook's
    Python functions) still run: nf_shutdown and every open batch at exit."""
    global _exit_registered, _live_batches
    if _exit_registered:
        return
    import atexit
    import weakref
    _live_batches = weakref.WeakSet()

    def release():
        for b in list(_live_batches):
            try:
                b.close()
            except Exception:
                pass
        if _lib is not None:
            _lib.nf_shutdown()
    atexit.register(release)
    _exit_registered = True


def last_error() -> str:
    return load().nf_last_error().decode("utf-8", "replace")


def _check(rc: int) -> int:
    if rc < 0:
        raise NFError(rc, last_error())
    return rc


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------- API

def nf_init(device: int = 0) -> None:
    _check(load().nf_init(device))


def nf_shutdown() -> None:
    load().nf_shutdown()


def nf_precompute_R(q: int) -> None:
    _check(load().nf_precompute_R(q))


def nf_copy_R(q: int) -> np.ndarray:
    size = 1 << (q - 1) if q >= 1 else 1
    out = np.zeros((size, size), dtype=np.uint8)
    _check(load().nf_copy_R(q, out.ctypes.data, out.nbytes))
    return out


def nf_fold(seq, q: int = 0, table: bool = False):
    """Fold one sequence; returns the score, or (score, table) with ``table``.

    The table is (n, n) int16 with T[i, j] = D(i+1, j+1) for i <= j, else 0.
    """
    b = seq.encode("ascii") if isinstance(seq, str) else bytes(seq)
    n = len(b)
    S = np.zeros((n, n), dtype=np.int16) if table else None
    score = _check(load().nf_fold(b, n, q, _ptr(S) if n else None))
    return (score, S) if table else score


def nf_fold_structure(seq, q: int = 0):
    """Fold one sequence; returns (score, structure) with the structure as a
    dot-bracket string (the traceback through D*, see nf.h)."""
    b = seq.encode("ascii") if isinstance(seq, str) else bytes(seq)
    n = len(b)
    out = ctypes.create_string_buffer(max(n, 1))
    score = _check(load().nf_fold_structure(b, n, q, out))
    return score, out.raw[:n].decode("ascii")


def _dev_ptr(x, dtype_name: str, min_numel: int, what: str):
    """Device address of a torch tensor argument, after checking that it is a
    contiguous device tensor of the right dtype holding at least min_numel
    elements (a raw integer address is passed through unchecked; None stays
    None)."""
    if x is None:
        return None
    if not hasattr(x, "data_ptr"):
        return int(x)
    import torch
    if not x.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    if x.dtype != getattr(torch, dtype_name):
        raise ValueError("%s must be %s, not %s" % (what, dtype_name, x.dtype))
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if x.numel() < min_numel:
        raise ValueError("%s holds %d elements, needs %d" % (what, x.numel(), min_numel))
    return x.data_ptr()


def _stream_handle(stream):
    if stream is not None and hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return stream


def nf_fold_dev(d_codes, n: int, q: int = 0, d_score=None, d_S=None, stream=None) -> None:
    """Asynchronous fold of device codes (torch uint8 tensor or raw pointer).

    Tensors are checked before the call: d_codes uint8 with >= n elements,
    d_score int32 with >= 1, d_S int16 with >= n*n; all contiguous, on the
    device."""
    if n < 0:
        raise ValueError("n must be >= 0")
    pc = _dev_ptr(d_codes, "uint8", n, "d_codes")
    ps = _dev_ptr(d_score, "int32", 1, "d_score")
    pS = _dev_ptr(d_S, "int16", n * n, "d_S")
    _check(load().nf_fold_dev(pc, n, q, ps, pS, _stream_handle(stream)))


def nf_fold_dev_noalloc(d_codes, n: int, q: int = 0, d_score=None, d_S=None, stream=None) -> None:
    """nf_fold_dev that allocates nothing: every buffer beyond the arguments
    lives in the library's static device scratch (n up to 3519 at q = 8).
    Same argument checks as nf_fold_dev."""
    if n < 0:
        raise ValueError("n must be >= 0")
    pc = _dev_ptr(d_codes, "uint8", n, "d_codes")
    ps = _dev_ptr(d_score, "int32", 1, "d_score")
    pS = _dev_ptr(d_S, "int16", n * n, "d_S")
    _check(load().nf_fold_dev_noalloc(pc, n, q, ps, pS, _stream_handle(stream)))


def nf_encode(seq) -> np.ndarray:
    """Base codes A=0, C=1, G=2, U=3 of a sequence, by the library
    (``nf_encode``), as ``nf_fold_dev`` takes them."""
    b = seq.encode("ascii") if isinstance(seq, str) else bytes(seq)
    out = np.zeros(max(1, len(b)), dtype=np.uint8)
    _check(load().nf_encode(b, len(b), out.ctypes.data))
    return out[: len(b)]


encode = nf_encode


class Batch:
    """A prepared batch (``nf_batch_*``): codes resident on the device and the
    whole packed-wavefront fill captured as one HIP graph."""

    def __init__(self, seqs: Sequence[str], q: int = 0):
        L = load()
        self._keep = [s.encode("ascii") for s in seqs]
        self.count = len(seqs)
        arr = (ctypes.c_char_p * max(1, self.count))(*self._keep)
        ns = (ctypes.c_int * max(1, self.count))(*[len(s) for s in self._keep])
        self.ns = [len(s) for s in self._keep]
        h = ctypes.c_void_p()
        self._h = None
        _check(L.nf_batch_create(ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(ns, ctypes.c_void_p),
                                 self.count, q, ctypes.byref(h)))
        self._h = h
        if _live_batches is not None:
            _live_batches.add(self)

    def run(self, stream=None) -> None:
        s = stream.cuda_stream if stream is not None and hasattr(stream, "cuda_stream") else stream
        _check(load().nf_batch_run(self._h, s))

    def scores(self) -> np.ndarray:
        out = np.zeros(max(1, self.count), dtype=np.int32)
        _check(load().nf_batch_scores(self._h, out.ctypes.data))
        return out[: self.count]

    def table(self, idx: int) -> np.ndarray:
        n = self.ns[idx]
        out = np.zeros((n, n), dtype=np.int16)
        _check(load().nf_batch_table(self._h, idx, out.ctypes.data if n else None))
        return out

    def structures(self) -> list:
        """One optimal dot-bracket structure per fold (nf_batch_structures)."""
        bufs = [ctypes.create_string_buffer(max(1, n)) for n in self.ns]
        ptrs = (ctypes.c_void_p * max(1, self.count))(*[ctypes.addressof(b) for b in bufs])
        _check(load().nf_batch_structures(self._h, ctypes.cast(ptrs, ctypes.c_void_p)))
        return [b.raw[:n].decode("ascii") for b, n in zip(bufs, self.ns)]

    def device_bytes(self) -> int:
        c = ctypes.c_int()
        b = ctypes.c_size_t()
        _check(load().nf_batch_info(self._h, ctypes.byref(c), ctypes.byref(b)))
        return b.value

    def close(self) -> None:
        if self._h:
            load().nf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nf_fold_batch(seqs: Sequence[str], q: int = 0, tables: bool = False):
    """Fold many sequences in one packed wavefront; scores (and tables)."""
    L = load()
    keep = [s.encode("ascii") for s in seqs]
    count = len(keep)
    arr = (ctypes.c_char_p * max(1, count))(*keep)
    ns = (ctypes.c_int * max(1, count))(*[len(s) for s in keep])
    scores = np.zeros(max(1, count), dtype=np.int32)
    S_list: List[np.ndarray] = []
    souts = None
    if tables:
        S_list = [np.zeros((len(s), len(s)), dtype=np.int16) for s in keep]
        souts = (ctypes.c_void_p * max(1, count))(*[x.ctypes.data if x.size else None for x in S_list])
    _check(L.nf_fold_batch(ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(ns, ctypes.c_void_p), count, q,
                           scores.ctypes.data, ctypes.cast(souts, ctypes.c_void_p) if souts is not None else None))
    return (scores[:count], S_list) if tables else scores[:count]


def nf_serve_config(hbm_budget_bytes: int = 0, max_slots: int = 0, max_queue: int = 0) -> None:
    _check(load().nf_serve_config(hbm_budget_bytes, max_slots, max_queue))


def nf_fold_bytes(n: int, q: int = 0) -> int:
    return int(load().nf_fold_bytes(n, q))


def nf_submit(seq: str, q: int = 0, want_table: bool = False, want_structure: bool = False) -> int:
    b = seq.encode("ascii")
    flags = (NF_WANT_TABLE if want_table else 0) | (NF_WANT_STRUCTURE if want_structure else 0)
    return _check(load().nf_submit(b, len(b), q, flags))


def nf_poll(ticket: int, n: int = 0, want_table: bool = False):
    """(done, score, table): done is False while the fold is pending."""
    score = ctypes.c_int32(-1)
    S = np.zeros((n, n), dtype=np.int16) if want_table else None
    rc = _check(load().nf_poll(ticket, ctypes.addressof(score), _ptr(S) if (S is not None and n) else None))
    return (rc == 1, score.value if rc == 1 else None, S if rc == 1 else None)


def nf_wait(ticket: int, timeout_ms: int = -1, n: int = 0, want_table: bool = False):
    score = ctypes.c_int32(-1)
    S = np.zeros((n, n), dtype=np.int16) if want_table else None
    _check(load().nf_wait(ticket, timeout_ms, ctypes.addressof(score), _ptr(S) if (S is not None and n) else None))
    return (score.value, S) if want_table else score.value


def nf_poll_ex(ticket: int, timeout_ms: int = -1, n: int = 0, want_table: bool = False,
               want_structure: bool = False):
    """(done, score, table, structure); timeout_ms 0 polls, < 0 waits without limit."""
    score = ctypes.c_int32(-1)
    S = np.zeros((n, n), dtype=np.int16) if want_table else None
    db = ctypes.create_string_buffer(max(1, n)) if want_structure else None
    rc = _check(load().nf_poll_ex(ticket, timeout_ms, ctypes.addressof(score),
                                  _ptr(S) if (S is not None and n) else None,
                                  ctypes.addressof(db) if db is not None else None))
    if rc != 1:
        return (False, None, None, None)
    return (True, score.value, S, db.raw[:n].decode("ascii") if db is not None else None)


def nf_serve_stats() -> ServeStats:
    st = ServeStats()
    _check(load().nf_serve_stats(ctypes.byref(st)))
    return st


def nf_autotune_q(n: int) -> int:
    return _check(load().nf_autotune_q(n))


def nf_autotune_target(n: int, q: int = 0) -> int:
    """Between-group chunks per wavefront step of a single fold of length n at
    group width q (0: the q that q = 0 resolves to)."""
    return _check(load().nf_autotune_target(n, q))


def nf_autotune_wide(n: int, q: int = 0) -> bool:
    """Whether a single fold of length n at q runs the wide fused step."""
    return bool(_check(load().nf_autotune_wide(n, q)))


def nf_autotune(n: int, qmin: int = 4, qmax: int = 8, reps: int = 3) -> int:
    """Tune q, then the chunk target, at length n; returns the chosen q."""
    return _check(load().nf_autotune(n, qmin, qmax, reps))


def nf_profile_fold(d_codes, n: int, q: int = 0, reps: int = 1, stream=None) -> KernelProfile:
    """Per-kernel HIP-event timing of the fill of device codes (see nf.h)."""
    if n < 0:
        raise ValueError("n must be >= 0")
    p = _dev_ptr(d_codes, "uint8", n, "d_codes")
    out = KernelProfile()
    _check(load().nf_profile_fold(p, n, q, reps, _stream_handle(stream), ctypes.byref(out)))
    return out


def nf_lds_gather_rate(table_bytes: int = 16384, row_bytes: int = 0) -> float:
    """LDS 1-byte gathers per second the device sustains over a table of
    table_bytes (uniform offsets, or one row of row_bytes per wavefront load)."""
    out = ctypes.c_double()
    _check(load().nf_lds_gather_rate(table_bytes, row_bytes, ctypes.byref(out)))
    return out.value
