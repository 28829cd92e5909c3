"""CPU oracle for the Nussinov table and the Four-Russians lookup table R.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU path (``paper_1307_7820_amd``) and imports nothing from it.

* ``fold_table`` / ``fold_score``: the plain O(n^3) recurrence of Section 2
  (Eq. 1), computed by the C routine in ``nussinov.c``.
* ``r_table``: the preprocessing step of Section 3.1 that, for every pair of a
  horizontal difference vector v and a vertical difference vector v-bar,
  returns the largest running total max_k (V_k + Vbar_k) (Eq. 3).
* ``structure``: the traceback of Section 2 through D*, the argmax of Eq. 1,
  giving one optimal secondary structure in dot-bracket form.
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

    R pairs a horizontal difference vector v (entries 0 or 1) with a vertical
    one v-bar (entries 0 or -1) and holds the largest prefix total
    max_k (V_k + Vbar_k) of Eq. 3, where V_k and Vbar_k are the sums of the
    first k+1 entries.  Both vectors start with v_0 = v-bar_0 = 0, so only
    q-1 entries carry information: bit p-1 of ``h`` is v_p and bit p-1 of
    ``c`` is -v-bar_p (p = 1..q-1).  The result is ``R[h, c]`` of shape
    (2^(q-1), 2^(q-1)).

    Computed from that definition: the prefix sums of the bits of h and of c
    (with the empty prefix, k = 0, first), their difference, and its maximum
    over k.  ``with_index`` also returns the smallest maximising k, the index
    the paper's listing keeps with its strict '>' comparison.
    """
    if not (1 <= q <= 12):
        raise ValueError("q out of range")
    m = q - 1
    size = 1 << m
    words = np.arange(size, dtype=np.int64)
    bits = (words[:, None] >> np.arange(m, dtype=np.int64)[None, :]) & 1      # [word, p-1]
    prefix = np.zeros((size, q), dtype=np.int16)                              # [word, k], k = 0..q-1
    prefix[:, 1:] = np.cumsum(bits, axis=1)
    # V_k + Vbar_k for every (h, c, k): prefix of h's bits minus prefix of c's
    totals = prefix[:, None, :] - prefix[None, :, :]
    R = totals.max(axis=2).astype(np.uint8)
    if with_index:
        return R, np.argmax(totals, axis=2).astype(np.uint8)  # argmax: first maximum
    return R


_PAIRS = {("A", "U"), ("U", "A"), ("C", "G"), ("G", "C")}


def structure(seq: str, table=None) -> str:
    """One optimal secondary structure of ``seq`` as a dot-bracket string.

    Section 2 keeps, beside each D(i, j), the indices D*(i, j) that attain the
    maximum (argmax in place of max in Eq. 1) and reads the structure back from
    D(1, n).  The argmax here is taken as a strict '>' scan takes it: the
    first maximising term in the order of Eq. 1, i.e. the pairing term
    b(S_i, S_j) + D(i+1, j-1) first, then the splits D(i, k) + D(k+1, j) for
    k = i, ..., j-1.  When the pairing term wins and S_i, S_j are
    complementary they form a pair; with b = 0 both stay unpaired.  D* is
    recomputed from the finished table on the way back instead of stored.

    ``table`` is ``fold_table(seq)`` if already computed (T[i-1, j-1] = D(i, j)).
    """
    n = len(seq)
    T = fold_table(seq) if table is None else np.asarray(table)
    s = seq.upper()

    def D(i: int, j: int) -> int:  # 1-based; D(i, i-1) = D(i, i) = 0
        return int(T[i - 1, j - 1]) if j > i else 0

    out = ["."] * n
    todo = [(1, n)] if n >= 2 else []
    while todo:
        i, j = todo.pop()
        while j - i >= 1:  # at least two bases
            v = D(i, j)
            b = 1 if (s[i - 1], s[j - 1]) in _PAIRS else 0
            if v == b + D(i + 1, j - 1):
                if b:
                    out[i - 1], out[j - 1] = "(", ")"
                i, j = i + 1, j - 1
                continue
            # D(i, k) for k = i..j-1 is row i-1 of T, columns i-1..j-2 (D(i, i) = 0
            # sits on the diagonal); D(k+1, j) is column j-1, rows i..j-1
            splits = T[i - 1, i - 1:j - 1].astype(np.int64) + T[i:j, j - 1].astype(np.int64)
            hits = np.flatnonzero(splits == v)
            if hits.size == 0:
                raise AssertionError("no term of Eq. 1 attains D(%d, %d)" % (i, j))
            k = i + int(hits[0])
            todo.append((k + 1, j))
            j = k
    return "".join(out)
