"""Pins for the CPU oracle (Eq. 1 of Section 2 and the R table of Section 3.1).

The oracle is trusted only because these tests tie it to things other than
itself: brute-force enumeration of non-crossing matchings, hand-worked tables,
a closed form for two-letter sequences, Lemma 1, symmetries of the problem,
and, for R, closed forms, a reflection-principle count and a direct
maximisation over explicit table values (Eq. 2 against Eq. 3).
"""

import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen
from pins import (au_closed_form_table, brute_force_max, brute_force_table, check_structure,
                  composition_upper_bound, lemma1_violations, reverse_table)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(path):
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([0 if t == "." else int(t) for t in line.split()])
    return np.array(rows, dtype=np.int32)


# ---------------------------------------------------------------- Eq. 1 pins

def test_hand_cases():
    for line in open(os.path.join(GOLDEN, "hand_cases.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        s, v = line.split()
        s = "" if s == "-" else s
        assert oracle.fold_score(s) == int(v), s
        assert brute_force_max(s) == int(v), s


@pytest.mark.parametrize("name", ["GGAUCC", "ACUGAUGC"])
def test_hand_tables(name):
    want = _read_table(os.path.join(GOLDEN, "table_%s.txt" % name))
    got = oracle.fold_table(name)
    assert np.array_equal(got, want)
    assert np.array_equal(brute_force_table(name), want)


def test_brute_force_every_cell_random():
    # every cell of every table: each substring enumerated independently
    for t in range(40):
        n = 4 + (t % 9)          # 4..12
        s = gen.iid_sequence(n, [7, t])
        assert np.array_equal(oracle.fold_table(s), brute_force_table(s)), s


def test_brute_force_n14():
    for t in range(3):
        s = gen.iid_sequence(14, [14, t])
        assert oracle.fold_score(s) == brute_force_max(s), s
    # worst case for the enumeration: 7 A and 7 U
    s = gen.iid_sequence(14, [15, 0], probs=(0.5, 0.0, 0.0, 0.5))
    assert oracle.fold_score(s) == brute_force_max(s), s


def test_exhaustive_small_alphabet_strings():
    # every string over A,C,G,U up to length 6: full table for n <= 4, score for all
    for n in range(0, 7):
        for tup in itertools.product("ACGU", repeat=n):
            s = "".join(tup)
            if n <= 4:
                assert np.array_equal(oracle.fold_table(s), brute_force_table(s)), s
            else:
                assert oracle.fold_score(s) == brute_force_max(s), s


@pytest.mark.parametrize("n,alpha,seed", [(300, "AU", 1), (777, "CG", 2), (1500, "AU", 3)])
def test_two_letter_closed_form(n, alpha, seed):
    p = (0.5, 0.0, 0.0, 0.5) if alpha == "AU" else (0.0, 0.5, 0.5, 0.0)
    s = gen.iid_sequence(n, [21, seed], probs=p)
    assert np.array_equal(oracle.fold_table(s), au_closed_form_table(s))


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (63, 2), (200, 3), (500, 4)])
def test_lemma1_and_upper_bound(n, seed):
    s = gen.iid_sequence(n, [31, seed])
    T = oracle.fold_table(s)
    assert lemma1_violations(T) == 0
    ub = composition_upper_bound(s)
    iu = np.triu(np.ones((n, n), dtype=bool))
    assert np.all(T[iu] <= ub[iu])
    assert np.all(T[iu] <= (np.arange(n)[None, :] - np.arange(n)[:, None] + 1)[iu] // 2)


def test_symmetries():
    s = gen.iid_sequence(257, [41, 0])
    T = oracle.fold_table(s)
    # reversal: D_rev(i, j) = D(n+1-j, n+1-i)
    assert np.array_equal(oracle.fold_table(s[::-1]), reverse_table(T))
    # complement A<->U, C<->G and the swap A<->C, U<->G both preserve b(.,.)
    comp = s.translate(str.maketrans("ACGU", "UGCA"))
    swap = s.translate(str.maketrans("ACGU", "CAUG"))
    assert np.array_equal(oracle.fold_table(comp), T)
    assert np.array_equal(oracle.fold_table(swap), T)


def test_planted_stem_sequence():
    # a perfect hairpin: stem of 30 bases, loop of 5 -> at least 30 pairs
    arm = gen.iid_sequence(30, [51, 0])
    s = arm + "AAAAA" + gen.reverse_complement(arm)
    assert oracle.fold_score(s) >= 30
    assert lemma1_violations(oracle.fold_table(s)) == 0


def test_lowercase_and_rejects():
    assert oracle.fold_score("gggaaaccc") == 3
    for bad in ["ACGT", "ACNU", "AC U", "AC-U"]:
        with pytest.raises(ValueError):
            oracle.fold_score(bad)


def test_thread_count_does_not_change_table():
    s = gen.iid_sequence(400, [61, 0])
    assert np.array_equal(oracle.fold_table(s, nthreads=1), oracle.fold_table(s, nthreads=4))


# ---------------------------------------------------------------- R table pins

def _popcount(x):
    return bin(int(x)).count("1")


@pytest.mark.parametrize("q", range(1, 10))
def test_r_closed_forms(q):
    R = oracle.r_table(q)
    m = q - 1
    size = 1 << m
    full = size - 1
    for h in range(size):
        assert R[h, 0] == _popcount(h)            # no drop down the column: all of v counts
        assert R[0, h] == 0                       # flat row: the running total never rises
        assert R[h, h] == 0                       # equal vectors cancel at every k
        assert R[full, h] == m - _popcount(h)     # rising row: total at k = q-1 is largest
    assert R.max() <= m


@pytest.mark.parametrize("q", range(1, 10))
def test_r_histogram_reflection_principle(q):
    # Mapping each (v_p, vbar_p) to two +-1 steps turns the running total into a
    # simple random walk of 2(q-1) steps watched at even times; the reflection
    # principle then gives #{R = r} = C(2q-1, q-1-r).
    R = oracle.r_table(q)
    counts = np.bincount(R.ravel(), minlength=q)
    for r in range(q):
        assert counts[r] == math.comb(2 * q - 1, q - 1 - r), (q, r)


def _staircase(rng, q, start, up):
    steps = rng.integers(0, 2, size=q - 1)
    vals = [start]
    for st in steps:
        vals.append(vals[-1] + (st if up else -st))
    return np.array(vals), steps


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_r_matches_direct_group_max(q):
    # Eq. 2 against Eq. 3: the max over q split points of row + column values
    # equals base_row + base_col + R[v][vbar] for explicit monotone vectors.
    R = oracle.r_table(q)
    rng = np.random.default_rng([71, q])
    for _ in range(2000):
        row, hs = _staircase(rng, q, int(rng.integers(0, 50)), up=True)    # D(i, l..l+q-1)
        col, cs = _staircase(rng, q, int(rng.integers(0, 50)), up=False)   # D(l+1..l+q, j)
        h = sum(int(b) << p for p, b in enumerate(hs))
        c = sum(int(b) << p for p, b in enumerate(cs))
        direct = int(np.max(row + col))
        assert direct == row[0] + col[0] + int(R[h, c])


def test_r_index_is_first_argmax():
    R, idx = oracle.r_table(6, with_index=True)
    m = 5
    for h in range(1 << m):
        for c in range(1 << m):
            tot = [0]
            for k in range(1, m + 1):
                tot.append(tot[-1] + ((h >> (k - 1)) & 1) - ((c >> (k - 1)) & 1))
            assert idx[h, c] == int(np.argmax(tot))
            assert R[h, c] == max(tot)


# ---------------------------------------------------------------- traceback pins
# The traceback of Section 2 (D*, the argmax of Eq. 1) read back from the
# oracle's table: pinned by hand-worked structures, by brute-force optimality
# and by the two-letter closed form.

def _golden_structures():
    for line in open(os.path.join(GOLDEN, "structures.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        seq, db = line.split()
        yield ("" if seq == "-" else seq), ("" if db == "-" else db)


def test_structure_hand_cases():
    for seq, db in _golden_structures():
        assert oracle.structure(seq) == db, seq


def test_structure_optimal_against_brute_force():
    rng = np.random.default_rng([201])
    for t in range(120):
        n = int(rng.integers(0, 13))
        seq = "".join(rng.choice(list("ACGU"), size=n))
        check_structure(seq, oracle.structure(seq), brute_force_max(seq))


def test_structure_valid_random_lengths():
    for t, n in enumerate([2, 3, 17, 64, 65, 200, 401]):
        seq = gen.iid_sequence(n, [202, t])
        T = oracle.fold_table(seq)
        check_structure(seq, oracle.structure(seq, T), int(T[0, -1]))


def test_structure_two_letter_closed_form():
    rng = np.random.default_rng([203])
    for t in range(20):
        n = int(rng.integers(1, 160))
        seq = "".join(rng.choice(list("AU"), size=n))
        check_structure(seq, oracle.structure(seq), min(seq.count("A"), seq.count("U")))
