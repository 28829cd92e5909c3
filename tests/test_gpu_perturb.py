"""Race detection by schedule perturbation (nf_test_set_perturb).

The tiles of one anti-diagonal are independent (Section 4), the between
chunks that share a tile's accumulator combine by atomic max, and the fused
step's finishes and between chunks touch disjoint data.  So the items of a
step may run in any order and overlap in any way.  Under several seeds every
step's items are shuffled (other workgroups, CUs and XCDs take them) and the
staged steps' launches on the two streams are delayed by different amounts;
every table must still equal the oracle's bit for bit, and the run without
perturbation.
"""

import os

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen

pytestmark = pytest.mark.gpu

SEEDS = [1, 2, 3]


@pytest.fixture(params=["staged", "fused"])
def nf_mode(request):
    from paper_1307_7820_amd import nf as m
    old = os.environ.get("NF_MODE")
    os.environ["NF_MODE"] = request.param
    m.nf_shutdown()
    yield m
    m.load().nf_test_set_perturb(0)
    m.nf_shutdown()
    if old is None:
        os.environ.pop("NF_MODE", None)
    else:
        os.environ["NF_MODE"] = old


def test_single_folds_under_perturbed_schedules(nf_mode):
    lib = nf_mode.load()
    cases = [(gen.iid_sequence(700, [1307, 90]), 8), (gen.stem_sequence(2000, [1307, 91]), 8),
             (gen.iid_sequence(1000, [1307, 92]), 5), (gen.workload_n6000(), 8)]
    want = [oracle.fold_table(s) for s, _ in cases]
    lib.nf_test_set_perturb(0)
    plain = [nf_mode.nf_fold(s, q=q, table=True)[1] for s, q in cases]
    for seed in SEEDS:
        print("perturbed single folds: mode=%s seed=%d" % (os.environ["NF_MODE"], seed), flush=True)
        assert lib.nf_test_set_perturb(seed) == 0
        for (s, q), w, p in zip(cases, want, plain):
            score, T = nf_mode.nf_fold(s, q=q, table=True)
            assert np.array_equal(T, w), (os.environ["NF_MODE"], seed, len(s), q)
            assert np.array_equal(T, p)
    lib.nf_test_set_perturb(0)


def test_batch_under_perturbed_schedules(nf_mode):
    lib = nf_mode.load()
    seqs = gen.batch_sequences(300, 50, 2000, (1307, 93))
    want = np.array([oracle.fold_score(s) for s in seqs], dtype=np.int32)
    longest = int(np.argmax([len(s) for s in seqs]))
    want_T = oracle.fold_table(seqs[longest])
    for seed in SEEDS:
        print("perturbed batch: mode=%s seed=%d" % (os.environ["NF_MODE"], seed), flush=True)
        assert lib.nf_test_set_perturb(seed) == 0
        b = nf_mode.Batch(seqs, q=8)
        for rep in range(2):  # the graph replayed
            b.run()
            got = b.scores()
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (seed, rep, bad[:10].tolist())
        assert np.array_equal(b.table(longest), want_T), seed
        b.close()
    lib.nf_test_set_perturb(0)
