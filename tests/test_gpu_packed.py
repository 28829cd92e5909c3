"""The packed state of every finished tile against words derived from the
oracle's table (the row and column difference vectors of Section 3.1, with
Lemma 1's 0/1 differences), read back through nf_test_packed_state.

For tile (A, B), row a and group k of its columns, the row word holds the
base F(a, BT+kq) in its low half and h << (q-1) above it, bit p-1 of h being
F(a, BT+kq+p) - F(a, BT+kq+p-1); for column b and group k of its rows, the
column word holds F(AT+kq, b) in its low half and c in its high half, bit
p-1 of c being F(AT+kq+p-1, b) - F(AT+kq+p, b).  F(a, b) = D(a+1, b), posts
past n taken from the sequence padded with 'A'.  Rows and columns at or past
T = (64/q)q are zero words.  Every word of every off-diagonal tile is
compared, including those no later step reads (the last diagonal's, the
padding), and the same workspace first holds another fold's state, so a word
the fill failed to write would show that fold's value.
"""

import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen

pytestmark = pytest.mark.gpu


def _post_table(seq, ld):
    """F(a, b) for posts 0..ld-1 of seq padded with 'A' to ld - 1 bases."""
    ext = seq + "A" * (ld - 1 - len(seq))
    D = oracle.fold_table(ext)  # D[i, j] = D(i+1, j+1), zero below the diagonal
    F = np.zeros((ld, ld), dtype=np.int64)
    F[: ld - 1, 1:] = D  # F(a, b) = D(a+1, b) = D[a, b-1]; zero for b <= a
    return F


def _expected_blocks(F, q, A, B):
    G = 64 // q
    T = G * q
    sub = F[A * T:A * T + T, B * T:B * T + T]
    w = np.array([1 << (p - 1) for p in range(1, q)], dtype=np.int64)
    # rows: groups of q columns
    g = sub.reshape(T, G, q)
    dr = g[:, :, 1:] - g[:, :, :-1]
    assert dr.min(initial=0) >= 0 and dr.max(initial=0) <= 1  # Lemma 1 along rows
    h = dr @ w if q > 1 else np.zeros((T, G), dtype=np.int64)
    row = np.zeros((G, 64), dtype=np.int64)
    row[:, :T] = (((h << (q - 1)) << 16) | g[:, :, 0]).T
    # columns: groups of q rows
    c3 = sub.reshape(G, q, T)
    dc = c3[:, :-1, :] - c3[:, 1:, :]
    assert dc.min(initial=0) >= 0 and dc.max(initial=0) <= 1  # Lemma 1 down columns
    c = np.einsum("gpt,p->gt", dc, w) if q > 1 else np.zeros((G, T), dtype=np.int64)
    col = np.zeros((G, 64), dtype=np.int64)
    col[:, :T] = (c << 16) | c3[:, 0, :]
    return row.astype(np.uint32), col.astype(np.uint32)


def _packed(nf, seq, q):
    lib = nf.load()
    nt = ctypes.c_int(0)
    probe = (ctypes.c_uint32 * 1)()
    lib.nf_test_packed_state(seq.encode(), len(seq), q, probe, probe, ctypes.c_size_t(0), ctypes.byref(nt))
    NT = nt.value
    words = NT * (NT + 1) // 2 * (64 // q) * 64
    rs = np.zeros(words, dtype=np.uint32)
    cs = np.zeros(words, dtype=np.uint32)
    score = lib.nf_test_packed_state(seq.encode(), len(seq), q, rs.ctypes.data_as(ctypes.c_void_p),
                                     cs.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(words),
                                     ctypes.byref(nt))
    assert score >= 0, nf.last_error()
    return score, NT, rs, cs


def _check(nf, seq, q, other_seed):
    G = 64 // q
    T = G * q
    # the same workspace first holds another sequence's state
    _packed(nf, gen.iid_sequence(len(seq), other_seed), q)
    score, NT, rs, cs = _packed(nf, seq, q)
    F = _post_table(seq, NT * T)
    assert score == F[0, len(seq)]
    blk = G * 64
    for d in range(1, NT):
        for A in range(NT - d):
            ti = d * NT - d * (d - 1) // 2 + A
            want_r, want_c = _expected_blocks(F, q, A, A + d)
            got_r = rs[ti * blk:(ti + 1) * blk].reshape(G, 64)
            got_c = cs[ti * blk:(ti + 1) * blk].reshape(G, 64)
            assert np.array_equal(got_r, want_r), ("row words", len(seq), q, A, d,
                                                   np.argwhere(got_r != want_r)[:4].tolist())
            assert np.array_equal(got_c, want_c), ("column words", len(seq), q, A, d,
                                                   np.argwhere(got_c != want_c)[:4].tolist())


@pytest.fixture(params=["staged", "fused"])
def nf(request):
    from paper_1307_7820_amd import nf as m
    old = os.environ.get("NF_MODE")
    os.environ["NF_MODE"] = request.param
    m.nf_shutdown()
    yield m
    m.nf_shutdown()
    if old is None:
        os.environ.pop("NF_MODE", None)
    else:
        os.environ["NF_MODE"] = old


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_packed_state_every_q(nf, q):
    print("packed state q=%d mode=%s" % (q, os.environ["NF_MODE"]), flush=True)
    for k, n in enumerate([2, 64, 333]):
        _check(nf, gen.iid_sequence(n, [1307, 80, q, k]), q, [1307, 81, q, k])
    _check(nf, gen.stem_sequence(520, [1307, 82, q]), q, [1307, 83, q])


def test_packed_state_long_fold(nf):
    print("packed state n=1283 q=8 mode=%s" % os.environ["NF_MODE"], flush=True)
    _check(nf, gen.iid_sequence(1283, [1307, 84]), 8, [1307, 85])


def test_packed_state_n6000_as_benched():
    """The headline fold in the launch configuration the benchmark times
    (fused steps, tuned q = 8): every packed word of its 4371 off-diagonal
    tiles."""
    from paper_1307_7820_amd import nf as m
    m.nf_shutdown()
    print("packed state n=6000 q=8", flush=True)
    _check(m, gen.workload_n6000(), 8, [1307, 86])
    m.nf_shutdown()
