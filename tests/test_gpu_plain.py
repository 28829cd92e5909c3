"""GPU parity of the plain between-group kernel (NF_BETWEEN=plain), the
ablation of the Four-Russians lookup: the between-group maxima come from the
dense table by Eq. 1's splits with no R, and every table must still equal the
oracle's, bit for bit."""

import os

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nf():
    old = os.environ.get("NF_BETWEEN")
    os.environ["NF_BETWEEN"] = "plain"
    from paper_1307_7820_amd import nf as m
    m.nf_init(0)
    yield m
    if old is None:
        os.environ.pop("NF_BETWEEN", None)
    else:
        os.environ["NF_BETWEEN"] = old


@pytest.mark.parametrize("q", [1, 2, 4, 8])
def test_tables_equal_oracle(nf, q):
    # several tile diagonals so chunks of one, two and many tiles C occur
    for k, n in enumerate([2, 65, 200, 320, 511, 700]):
        s = gen.iid_sequence(n, [501, q, k])
        score, T = nf.nf_fold(s, q=q, table=True)
        assert np.array_equal(T, oracle.fold_table(s)), (q, n)


def test_structured_and_two_letter(nf):
    for t, s in enumerate([gen.stem_sequence(900, [502, 0]), "A" * 300 + "U" * 300, "GC" * 260]):
        score, T = nf.nf_fold(s, q=8, table=True)
        assert np.array_equal(T, oracle.fold_table(s)), t


def test_n6000_table(nf):
    s = gen.workload_n6000()
    score, T = nf.nf_fold(s, q=8, table=True)
    assert np.array_equal(T, oracle.fold_table(s))


def test_plain_runs_staged_steps(nf):
    # NF_BETWEEN=plain makes a new workspace that runs staged steps (the fused
    # step has the lookup built in): between launches, no fused launches,
    # although a single fold would otherwise run fused steps
    import torch
    s = gen.iid_sequence(3000, [503, 0])
    codes = torch.from_numpy(nf.encode(s)).cuda()
    prof = nf.nf_profile_fold(codes, len(s), 8, 1)
    assert prof.launches[2] > 0 and prof.launches[3] == 0
    os.environ.pop("NF_BETWEEN")
    try:
        prof = nf.nf_profile_fold(codes, len(s), 8, 1)
        assert prof.launches[3] > 0  # the lookup workspace for the same (n, q)
    finally:
        os.environ["NF_BETWEEN"] = "plain"
