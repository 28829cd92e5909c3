"""ctypes binding of libnf_serial.so (include/nf_serial.h): the paper's
serial CPU algorithms of Section 3, for its serial comparisons (Section 6).

Host code only, and a library of its own: the GPU path (``nf``) never calls
it.  Names and arguments as in the C ABI.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnf_serial.so")

NF_SERIAL_PLAIN = 0
NF_SERIAL_TWO_VECTOR = 1
NF_SERIAL_PARTIAL_MEMO = 2
NF_SERIAL_FULL_MEMO = 3
NF_SERIAL_FG = 4
VARIANTS = {"plain": NF_SERIAL_PLAIN, "two_vector": NF_SERIAL_TWO_VECTOR,
            "partial_memo": NF_SERIAL_PARTIAL_MEMO, "full_memo": NF_SERIAL_FULL_MEMO, "fg": NF_SERIAL_FG}


class SerialStats(ctypes.Structure):
    _fields_ = [("lookups", ctypes.c_int64), ("splits", ctypes.c_int64),
                ("r_entries", ctypes.c_int64), ("vectors", ctypes.c_int64)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libnf_serial.so not found at %s; build it with "
                              "`python -m paper_1307_7820_amd.build`" % path)
        L = ctypes.CDLL(path)
        L.nf_serial_fold.restype = ctypes.c_int
        L.nf_serial_fold.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.POINTER(SerialStats)]
        _lib = L
    return _lib


def nf_serial_fold(seq: str, q: int = 8, variant="two_vector", threads: int = 1, table: bool = False):
    """Fold on the host by one of the paper's serial algorithms.

    Returns (score, stats) or (score, stats, table); the table is (n, n) int16
    with T[i, j] = D(i+1, j+1) for i <= j, else 0."""
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    b = seq.encode("ascii")
    n = len(b)
    S = np.zeros((n, n), dtype=np.int16) if table else None
    st = SerialStats()
    rc = load().nf_serial_fold(b, n, q, v, threads, S.ctypes.data if (S is not None and n) else None,
                               ctypes.byref(st))
    if rc == -1:
        raise ValueError("nf_serial_fold: bad argument or base")
    if rc == -2:
        raise MemoryError("nf_serial_fold: host memory")
    return (rc, st, S) if table else (rc, st)
