"""The paper's serial CPU algorithms (libnf_serial.so, Section 3): Algorithm 1
(two-vector), the partially and completely memoized variants, Frid-Gusfield
and the plain recurrence, in column order and, for two-vector and plain, in
multicore anti-diagonal order.  Every one must give the table of Eq. 1
exactly (the oracle's), and the work it reports must cover every split point
of every cell exactly once."""

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen, serial

VARIANTS = ["plain", "two_vector", "partial_memo", "full_memo", "fg"]


def _cases():
    out = [("", 0), ("A", 1), ("AU", 2), ("GGGAAACCC", 3), ("ACUGAUGC", 4)]
    rng = np.random.default_rng([1307, 70])
    for t in range(12):
        n = int(rng.integers(3, 160))
        out.append((gen.iid_sequence(n, [1307, 71, t]), 10 + t))
    out.append((gen.stem_sequence(150, [1307, 72]), 30))
    out.append((gen.iid_sequence(120, [1307, 73], probs=(0.5, 0.0, 0.0, 0.5)), 31))
    return out


@pytest.mark.parametrize("variant", VARIANTS)
def test_every_variant_and_q_gives_the_oracle_table(variant):
    qs = [1] if variant == "plain" else list(range(1, 10))
    for s, _ in _cases():
        want = oracle.fold_table(s).astype(np.int16)
        for q in qs:
            for th in ([1, 4] if variant in ("plain", "two_vector") else [1]):
                score, st, T = serial.nf_serial_fold(s, q, variant, th, table=True)
                assert np.array_equal(T, want), (variant, q, th, len(s))
                assert score == (int(want[0, -1]) if s else 0)


@pytest.mark.parametrize("variant,q", [("two_vector", 8), ("partial_memo", 8), ("full_memo", 6), ("fg", 3)])
def test_n1000(variant, q):
    s = gen.iid_sequence(1000, [1307, 74])
    score, st, T = serial.nf_serial_fold(s, q, variant, table=True)
    assert np.array_equal(T, oracle.fold_table(s).astype(np.int16))


def test_multicore_two_vector_at_n2000():
    s = gen.iid_sequence(2000, [1307, 75])
    a = serial.nf_serial_fold(s, 8, "two_vector", 8, table=True)
    b = serial.nf_serial_fold(s, 8, "two_vector", 1, table=True)
    assert a[0] == b[0] == oracle.fold_score(s)
    assert np.array_equal(a[2], b[2])


def test_work_covers_every_split_exactly_once():
    s = gen.iid_sequence(700, [1307, 76])
    n = len(s)
    total = (n - 1) * n * (n + 1) // 6  # split points of Eq. 1 over the table
    _, st = serial.nf_serial_fold(s, 1, "plain")
    assert st.splits == total and st.lookups == 0
    for q in (2, 3, 5, 8, 9):
        looked = {}
        for v in VARIANTS[1:]:
            _, st = serial.nf_serial_fold(s, q, v)
            assert st.lookups * q + st.splits == total, (v, q)
            looked[v] = (st.lookups, st.splits, st.vectors, st.r_entries)
        assert len({x[:3] for x in looked.values()}) == 1  # same groups, same vectors
        S = 1 << (q - 1)
        assert looked["two_vector"][3] == S * S                       # every pair, up front
        assert looked["partial_memo"][3] % S == 0                     # whole rows of R
        assert looked["partial_memo"][3] <= S * S
        assert looked["full_memo"][3] <= min(S * S, looked["full_memo"][0])  # pairs met
        assert looked["fg"][3] > looked["two_vector"][3] or q <= 2     # FG redoes rows


def test_bad_arguments():
    with pytest.raises(ValueError):
        serial.nf_serial_fold("ACGT", 4)
    with pytest.raises(ValueError):
        serial.nf_serial_fold("ACGU", 0, "two_vector")
    with pytest.raises(ValueError):
        serial.nf_serial_fold("ACGU", 13, "two_vector")
    with pytest.raises(ValueError):
        serial.nf_serial_fold("ACGU", 4, "full_memo", threads=2)
    with pytest.raises(ValueError):
        serial.nf_serial_fold("ACGU", 4, 9)


def test_library_exports_every_declared_symbol():
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(root, "include", "nf_serial.h")).read(), flags=re.S)
    names = set(re.findall(r"\b(nf_serial_[A-Za-z_]+)\s*\(", text))
    assert names == {"nf_serial_fold"}
    lib = serial.load()
    for name in names:
        assert hasattr(lib, name), name
