"""Independent pins for the oracle: brute force, closed forms, invariants.

None of these reuse the recurrence of Eq. 1.  They restate the problem of
Section 2 directly (a matching is a set of disjoint complementary pairs, and
two pairs (i, j), (k, l) with i < k may only be nested, k < l < j, or disjoint,
j < k) and derive values from it by enumeration or by counting.
"""

from __future__ import annotations

import itertools
from typing import List

import numpy as np

_PAIRS = {("A", "U"), ("U", "A"), ("C", "G"), ("G", "C")}


def complementary(x: str, y: str) -> bool:
    return (x.upper(), y.upper()) in _PAIRS


def crosses(p, r) -> bool:
    """True when pairs p and r are neither nested nor disjoint (Section 2)."""
    (i, j), (k, l) = sorted([p, r])
    return i < k < j < l


def brute_force_max(seq: str) -> int:
    """Largest non-crossing matching, by enumerating matchings.

    Walks positions left to right; each free position is either left unpaired
    or paired with a later free complementary position.  A pair is only added
    when the explicit pairwise test says it crosses none of the pairs chosen so
    far.  Exponential; meant for n <= 14.
    """
    n = len(seq)
    best = 0
    chosen: List[tuple] = []
    used = [False] * n

    def rec(pos: int) -> None:
        nonlocal best
        while pos < n and used[pos]:
            pos += 1
        if pos >= n:
            best = max(best, len(chosen))
            return
        # upper bound: every remaining free position could at best pair once
        free = sum(1 for x in range(pos, n) if not used[x])
        if len(chosen) + free // 2 <= best:
            return
        used[pos] = True
        for j in range(pos + 1, n):
            if used[j] or not complementary(seq[pos], seq[j]):
                continue
            cand = (pos, j)
            if any(crosses(cand, p) for p in chosen):
                continue
            used[j] = True
            chosen.append(cand)
            rec(pos + 1)
            chosen.pop()
            used[j] = False
        used[pos] = False
        # leave pos unpaired: mark it used so the walk moves on
        used[pos] = True
        rec(pos + 1)
        used[pos] = False

    rec(0)
    return best


def brute_force_table(seq: str) -> np.ndarray:
    """Every cell D(i, j) by brute force over the substring S_i..S_j."""
    n = len(seq)
    T = np.zeros((n, n), dtype=np.int32)
    for i in range(n):
        for j in range(i, n):
            T[i, j] = brute_force_max(seq[i:j + 1])
    return T


def au_closed_form_table(seq: str) -> np.ndarray:
    """For sequences over {A, U} only (or {C, G} only): D(i, j) = min(#A, #U).

    Upper bound: each pair uses one A and one U.  Lower bound: while both
    letters remain, some adjacent pair of unequal letters exists; pairing it
    crosses nothing, and removing it leaves the same situation.
    """
    s = seq.upper()
    letters = set(s)
    if letters <= {"A", "U"}:
        x, y = "A", "U"
    elif letters <= {"C", "G"}:
        x, y = "C", "G"
    else:
        raise ValueError("sequence must be over {A,U} or over {C,G}")
    n = len(s)
    cx = np.concatenate([[0], np.cumsum([c == x for c in s])]).astype(np.int64)
    cy = np.concatenate([[0], np.cumsum([c == y for c in s])]).astype(np.int64)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    nx = cx[j + 1] - cx[i]
    ny = cy[j + 1] - cy[i]
    T = np.minimum(nx, ny)
    T[j < i] = 0
    return T.astype(np.int32)


def composition_upper_bound(seq: str) -> np.ndarray:
    """min(#A,#U) + min(#C,#G) over S_i..S_j: no matching can exceed it."""
    s = seq.upper()
    n = len(s)
    cnt = {}
    for ch in "ACGU":
        cnt[ch] = np.concatenate([[0], np.cumsum([c == ch for c in s])]).astype(np.int64)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]

    def c(ch):
        return cnt[ch][np.clip(j + 1, 0, n)] - cnt[ch][i]

    T = np.minimum(c("A"), c("U")) + np.minimum(c("C"), c("G"))
    T[j < i] = 0
    return T


def lemma1_violations(T: np.ndarray) -> int:
    """Count violations of Lemma 1 on an (n, n) table with T[i, j] = D(i+1, j+1).

    Along a row (left to right) and up a column (bottom to top) values never
    decrease and neighbours differ by at most 1; the boundary D(i, i-1) = 0
    counts as a neighbour of the diagonal.
    """
    n = T.shape[0]
    if n == 0:
        return 0
    T = T.astype(np.int64)
    bad = 0
    iu = np.triu(np.ones((n, n), dtype=bool))
    # row steps: D(i, j) - D(i, j-1) for j > i; the diagonal cell against D(i, i-1) = 0
    row = np.diff(T, axis=1)
    m_row = iu[:, 1:] & iu[:, :-1]
    bad += int(np.count_nonzero(((row < 0) | (row > 1)) & m_row))
    # column steps: D(i, j) - D(i+1, j) for i < j
    col = T[:-1, :] - T[1:, :]
    m_col = iu[:-1, :] & iu[1:, :]
    bad += int(np.count_nonzero(((col < 0) | (col > 1)) & m_col))
    diag = np.diag(T)
    bad += int(np.count_nonzero(diag != 0))
    return bad


def reverse_table(T: np.ndarray) -> np.ndarray:
    """Table of the reversed sequence: D_rev(i, j) = D(n+1-j, n+1-i)."""
    return T[::-1, ::-1].T.copy()


def structure_pairs(db: str) -> list:
    """Pairs (i, j), 0-based, of a dot-bracket string; AssertionError when the
    brackets do not match or a character is not one of '(', ')', '.'."""
    stack, pairs = [], []
    for x, ch in enumerate(db):
        if ch == "(":
            stack.append(x)
        elif ch == ")":
            assert stack, "')' at %d closes nothing" % x
            pairs.append((stack.pop(), x))
        else:
            assert ch == ".", "bad character %r at %d" % (ch, x)
    assert not stack, "'(' at %d is never closed" % stack[-1]
    return pairs


def check_structure(seq: str, db: str, score: int) -> None:
    """A structure is a set of non-crossing complementary pairs (Section 2);
    an optimal one has D(1, n) of them.  Matched brackets cannot cross; the
    pairwise test checks that independently."""
    assert len(db) == len(seq), (len(db), len(seq))
    pairs = structure_pairs(db)
    for i, j in pairs:
        assert complementary(seq[i], seq[j]), (i, j, seq[i], seq[j])
    for p, r in itertools.combinations(pairs[:200], 2):
        assert not crosses(p, r), (p, r)
    assert len(pairs) == score, (len(pairs), score)
