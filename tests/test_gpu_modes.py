"""GPU parity of both executions of the fill (staged and fused steps).

They run the same kernels' arithmetic in different launch structures, so
each must give the CPU oracle's table bit for bit.
"""

import os

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen

pytestmark = pytest.mark.gpu

MODES = ["staged", "fused"]


@pytest.fixture(params=MODES)
def nf_mode(request):
    from paper_1307_7820_amd import nf as m
    old = os.environ.get("NF_MODE")
    os.environ["NF_MODE"] = request.param
    m.nf_shutdown()  # drop cached workspaces so new ones take this mode
    yield m
    m.nf_shutdown()
    if old is None:
        os.environ.pop("NF_MODE", None)
    else:
        os.environ["NF_MODE"] = old


def test_every_q_ragged_sizes(nf_mode):
    for q in range(1, 9):
        for k, n in enumerate([63, 64, 65, 129, 257, 449]):
            s = gen.iid_sequence(n, [301, q, k])
            score, T = nf_mode.nf_fold(s, q=q, table=True)
            assert np.array_equal(T, oracle.fold_table(s)), (q, n)


def test_random_lengths(nf_mode):
    rng = np.random.default_rng([302])
    for t in range(12):
        n = int(rng.integers(2, 900))
        q = int(rng.integers(4, 9))
        s = gen.iid_sequence(n, [303, t])
        score, T = nf_mode.nf_fold(s, q=q, table=True)
        assert np.array_equal(T, oracle.fold_table(s)), (n, q)


def test_n6000_full_table(nf_mode):
    s = gen.workload_n6000()
    score, T = nf_mode.nf_fold(s, q=8, table=True)
    assert np.array_equal(T, oracle.fold_table(s))


def test_batch_equals_alone_and_oracle(nf_mode):
    rng = np.random.default_rng([304])
    seqs = [gen.iid_sequence(int(rng.integers(0, 1500)), [305, t]) for t in range(40)] + ["", "GC"]
    scores, tables = nf_mode.nf_fold_batch(seqs, q=8, tables=True)
    for s, sc, T in zip(seqs, scores, tables):
        assert np.array_equal(T, oracle.fold_table(s)), len(s)
        assert sc == nf_mode.nf_fold(s, q=8)


def test_repeat_runs_identical(nf_mode):
    # workspaces are reused across runs: counters and accumulators must be
    # back at zero after every run
    s1 = gen.iid_sequence(3000, [306, 0])
    s2 = gen.iid_sequence(3000, [306, 1])
    a = nf_mode.nf_fold(s1, q=8)
    b = nf_mode.nf_fold(s2, q=8)
    assert a == oracle.fold_score(s1)
    assert b == oracle.fold_score(s2)
    assert nf_mode.nf_fold(s1, q=8) == a


@pytest.fixture(params=["0", "1"])
def nf_shape(request):
    """Both shapes of the fused step (default and wide, q = 8), forced."""
    from paper_1307_7820_amd import nf as m
    old = {k: os.environ.get(k) for k in ("NF_STAGE_WIDE", "NF_MODE")}
    os.environ["NF_STAGE_WIDE"] = request.param
    os.environ["NF_MODE"] = "fused"
    m.nf_shutdown()
    yield m
    m.nf_shutdown()
    for k, v in old.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def test_fused_step_shapes_equal_the_oracle(nf_shape):
    wide = os.environ["NF_STAGE_WIDE"] == "1"
    for k, n in enumerate([2, 63, 64, 65, 255, 257, 700, 1283]):
        s = gen.iid_sequence(n, [310, k])
        assert nf_shape.nf_autotune_wide(n, 8) == wide
        score, T = nf_shape.nf_fold(s, q=8, table=True)
        assert np.array_equal(T, oracle.fold_table(s)), (n, wide)
    s = gen.stem_sequence(900, [311])
    assert np.array_equal(nf_shape.nf_fold(s, q=8, table=True)[1], oracle.fold_table(s))
    # the headline length in the shape it does not take by default, and back
    s = gen.workload_n6000()
    score, T = nf_shape.nf_fold(s, q=8, table=True)
    assert np.array_equal(T, oracle.fold_table(s)), wide
