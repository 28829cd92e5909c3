"""CPU oracle for the Nussinov table and the Four-Russians lookup table R.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU path (``paper_1307_7820_amd``) and imports nothing from it.

* ``fold_table`` / ``fold_score``: the plain O(n^3) recurrence of Section 2
  (Eq. 1), computed by the C routine in ``nussinov.c``.
* ``r_table``: the preprocessing step of Section 3.1 that, for every pair of a
  horizontal difference vector v and a vertical difference vector v-bar,
  returns the largest running total max_k (V_k + Vbar_k) (Eq. 3).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nussinov.c")
_LIB = os.path.join(_HERE, "libnforacle.so")
_lock = threading.Lock()
_lib = None

# -march=x86-64-v3 (AVX2) rather than -march=native: the library is built in
# one container and may run on another host CPU.
CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile nussinov.c into libnforacle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            lib.nfo_fold.restype = ctypes.c_longlong
            lib.nfo_fold.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
            lib.nfo_max_threads.restype = ctypes.c_int
            lib.nfo_max_threads.argtypes = [ctypes.c_int]
            _lib = lib
    return _lib


def threads_used(nthreads: int = 0) -> int:
    """OpenMP thread count the oracle runs with for a given request (0 = default)."""
    return int(_load().nfo_max_threads(int(nthreads)))


def _check(rc: int) -> int:
    if rc == -1:
        raise ValueError("sequence holds a character outside A, C, G, U")
    if rc == -2:
        raise ValueError("negative length")
    if rc == -3:
        raise MemoryError("oracle could not allocate its table")
    return rc


def fold_table(seq: str, nthreads: int = 0) -> np.ndarray:
    """Full table of Eq. 1 as an (n, n) int32 array.

    ``T[i, j] = D(i+1, j+1)`` for i <= j (0-based array indices, 1-based D), and
    0 below the diagonal.
    """
    n = len(seq)
    out = np.zeros((n, n), dtype=np.int32)
    _check(_load().nfo_fold(seq.encode("ascii"), n, out.ctypes.data if n else None, int(nthreads)))
    return out


def fold_score(seq: str, nthreads: int = 0) -> int:
    """D(1, n) of Eq. 1 (0 for n <= 1)."""
    return int(_check(_load().nfo_fold(seq.encode("ascii"), len(seq), None, int(nthreads))))


def r_table(q: int, with_index: bool = False):
    """The table R of Section 3.1 for vectors of length q.

    The paper indexes R by the pair (v, v-bar) with v in {0,1}^q and v-bar in
    {0,-1}^q, where v_0 = v-bar_0 = 0 by definition, so only q-1 entries carry
    information.  Here both vectors are encoded by their informative entries:
    bit p-1 of ``h`` is v_p and bit p-1 of ``c`` is -v-bar_p (p = 1..q-1), and
    the result is an array ``R[h, c]`` of shape (2^(q-1), 2^(q-1)).

    Each entry follows the preprocessing listing: running sums of v and of
    v-bar over k = 0..q-1, keeping the largest sum total (starting from 0) and,
    with ``with_index``, the first k at which it is reached (strict '>').
    """
    if not (1 <= q <= 12):
        raise ValueError("q out of range")
    m = q - 1
    size = 1 << m
    h = np.arange(size, dtype=np.int64)[:, None] * np.ones((1, size), dtype=np.int64)
    c = np.ones((size, 1), dtype=np.int64) * np.arange(size, dtype=np.int64)[None, :]
    max_val = np.zeros((size, size), dtype=np.int64)
    max_idx = np.zeros((size, size), dtype=np.int64)
    sum1 = np.zeros((size, size), dtype=np.int64)
    sum2 = np.zeros((size, size), dtype=np.int64)
    for k in range(q):
        if k >= 1:
            v_k = (h >> (k - 1)) & 1           # horizontal difference v_k in {0, 1}
            vbar_k = -((c >> (k - 1)) & 1)     # vertical difference v-bar_k in {0, -1}
        else:
            v_k = np.zeros_like(h)             # v_0 = 0
            vbar_k = np.zeros_like(c)          # v-bar_0 = 0
        sum1 = sum1 + v_k
        sum2 = sum2 + vbar_k
        better = (sum1 + sum2) > max_val
        max_val = np.where(better, sum1 + sum2, max_val)
        max_idx = np.where(better, k, max_idx)
    R = max_val.astype(np.uint8)
    if with_index:
        return R, max_idx.astype(np.uint8)
    return R
