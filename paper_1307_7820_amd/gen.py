"""Seeded synthetic RNA inputs shared by the tests, the benchmark and the smoke check.

This module holds no part of the folding arithmetic: it only draws sequences over
the alphabet {A, C, G, U} (Section 2) with the shapes of the workloads the
benchmark reports on.  The paper measured on mouse non-coding RNA, on random
substrings of real RNA and on random A/C/G/U strings (Section 6); only the last
kind can be produced here, so GC-biased sequences with planted inverted repeats
stand in for structured real RNA.

Every generator takes an explicit seed (an int or a list of ints, passed to
``numpy.random.default_rng``) and returns plain Python ``str`` objects, so the
same call always returns the same inputs on every machine.
"""

from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

ALPHABET = "ACGU"
_WC = {"A": "U", "U": "A", "C": "G", "G": "C"}


def _rng(seed) -> np.random.Generator:
    return np.random.default_rng(seed)


def iid_sequence(n: int, seed, probs: Sequence[float] = (0.25, 0.25, 0.25, 0.25)) -> str:
    """n bases drawn iid over A, C, G, U with the given probabilities."""
    if n < 0:
        raise ValueError("n must be >= 0")
    rng = _rng(seed)
    idx = rng.choice(4, size=n, p=np.asarray(probs, dtype=np.float64))
    return "".join(ALPHABET[i] for i in idx)


def reverse_complement(s: str) -> str:
    """Watson-Crick reverse complement (A<->U, C<->G), read backwards."""
    return "".join(_WC[c] for c in reversed(s))


def stem_sequence(n: int, seed, gc: float = 0.60, stem_len=(20, 40), loop_len=(3, 200),
                  stems_per_base: float = 0.4 / 60.0) -> str:
    """GC-biased background with planted inverted repeats (hairpin stems).

    Background: P(G) = P(C) = gc/2, P(A) = P(U) = (1-gc)/2.  Then
    K = round(stems_per_base * n) stems are planted one after the other: a stem
    length L ~ U{stem_len}, a loop length l ~ U{loop_len} and a start p uniform
    over the positions where 2L + l bases fit; the reverse complement of
    S[p:p+L] is written at p+L+l.  Later stems overwrite earlier ones.
    """
    rng = _rng(seed)
    p_at = (1.0 - gc) / 2.0
    p_gc = gc / 2.0
    idx = rng.choice(4, size=n, p=np.array([p_at, p_gc, p_gc, p_at]))
    s = [ALPHABET[i] for i in idx]
    k = int(round(stems_per_base * n))
    for _ in range(k):
        L = int(rng.integers(stem_len[0], stem_len[1] + 1))
        l = int(rng.integers(loop_len[0], loop_len[1] + 1))
        span = 2 * L + l
        if span > n:
            continue
        p = int(rng.integers(0, n - span + 1))
        arm = "".join(s[p:p + L])
        rc = reverse_complement(arm)
        s[p + L + l:p + L + l + L] = list(rc)
    return "".join(s)


def loguniform_lengths(count: int, lo: int, hi: int, seed) -> List[int]:
    """count lengths n = round(exp(U(ln lo, ln hi)))."""
    rng = _rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return [int(round(math.exp(x))) for x in u]


def batch_sequences(count: int = 4096, lo: int = 50, hi: int = 2000, seed=(1307, 4)) -> List[str]:
    """A batch of iid uniform sequences with log-uniform lengths in [lo, hi]."""
    rng = _rng(list(seed) if not isinstance(seed, int) else seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    lens = [int(round(math.exp(x))) for x in u]
    out = []
    for n in lens:
        idx = rng.integers(0, 4, size=n)
        out.append("".join(ALPHABET[i] for i in idx))
    return out


def serving_trace(count: int, rate_per_s: float, seed=(1307, 5), short=(100, 500),
                  long=(2000, 8000), p_short: float = 0.8) -> List[Tuple[float, str]]:
    """Poisson arrivals at a fixed offered rate with a bimodal length mix.

    Returns (arrival_time_s, sequence) pairs sorted by time.  Lengths are
    U{short} with probability p_short and U{long} otherwise; bases iid uniform.
    """
    rng = _rng(list(seed) if not isinstance(seed, int) else seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate_per_s)) if rate_per_s > 0 else 0.0
        if rng.uniform() < p_short:
            n = int(rng.integers(short[0], short[1] + 1))
        else:
            n = int(rng.integers(long[0], long[1] + 1))
        idx = rng.integers(0, 4, size=n)
        out.append((t, "".join(ALPHABET[i] for i in idx)))
    return out


# Named workloads (sizes and structure of the reported configurations).

def workload_n500() -> str:
    """Single iid uniform sequence, n = 500."""
    return iid_sequence(500, [1307, 1])


def workload_n6000() -> str:
    """Single iid uniform sequence, n = 6000."""
    return iid_sequence(6000, [1307, 2])


def workload_n16000() -> str:
    """Single n = 16000 sequence, 60 % GC with planted stems of 20-40 bp."""
    return stem_sequence(16000, [1307, 3])


def workload_batch4096() -> List[str]:
    """4096 iid uniform sequences, lengths log-uniform in [50, 2000]."""
    return batch_sequences(4096, 50, 2000, (1307, 4))
