"""GPU parity at the sizes of the batch and serving workloads.

* The 4096-sequence batch (lengths log-uniform in [50, 2000]) in the launch
  configuration the benchmark times (one prepared batch, q = 8, staged steps
  captured as one graph): every score equals the oracle's (Eq. 1), and full
  tables equal the oracle's for the 32 longest folds and 32 drawn at random.
* A served mix with the serving workload's length bands (80% U{100..500},
  20% U{2000..8000}): every score, and the tables asked for, equal the
  oracle's and the same folds run alone.

Integer tables: every comparison is bit-exact.
"""

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture()
def nf():
    from paper_1307_7820_amd import nf as m
    m.nf_shutdown()
    yield m
    m.nf_shutdown()


def test_batch4096_every_score_and_sampled_tables(nf):
    seqs = gen.workload_batch4096()
    ns = np.array([len(s) for s in seqs])
    print("batch4096: %d folds, n %d..%d" % (len(seqs), ns.min(), ns.max()), flush=True)
    b = nf.Batch(seqs, q=8)
    b.run()
    got = b.scores()
    want = np.array([oracle.fold_score(s) for s in seqs], dtype=np.int32)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "scores differ at %s" % bad[:10].tolist()
    longest = np.argsort(-ns, kind="stable")[:32]
    rng = np.random.default_rng([1307, 40])
    drawn = rng.choice(len(seqs), size=32, replace=False)
    assert ns[longest].min() >= 1900
    for k in list(longest) + list(drawn):
        T = b.table(int(k))
        assert np.array_equal(T, oracle.fold_table(seqs[k])), (int(k), len(seqs[k]))
    # a second run of the same graph gives the same bits
    b.run()
    assert np.array_equal(b.scores(), want)
    b.close()


def test_serving_mix_with_long_band(nf):
    import time

    nf.nf_serve_config(2 << 30, 256, 0)  # the binding budget the benchmark serves under
    trace = gen.serving_trace(48, 0.0, seed=(1307, 5))
    seqs = [s for _, s in trace]
    long_idx = [k for k, s in enumerate(seqs) if len(s) >= 2000]
    assert len(long_idx) >= 6, len(long_idx)
    want_table = {k: (k in long_idx[::2]) or (len(seqs[k]) < 2000 and k % 7 == 0) for k in range(len(seqs))}
    print("serving mix: %d requests, %d long (n %s)" % (len(seqs), len(long_idx),
                                                         [len(seqs[k]) for k in long_idx]), flush=True)
    tickets = [nf.nf_submit(s, q=8, want_table=want_table[k]) for k, s in enumerate(seqs)]
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for k, t in enumerate(tickets):
            if k in res:
                continue
            done, score, S = nf.nf_poll(t, len(seqs[k]), want_table[k])
            if done:
                res[k] = (score, S)
        assert time.time() - t0 < 300, "serving did not finish"
        time.sleep(0.001)
    st = nf.nf_serve_stats()
    assert st.completed == len(seqs)
    assert st.peak_bytes <= 2 << 30
    nf.nf_shutdown()
    for k, s in enumerate(seqs):
        score, S = res[k]
        if want_table[k]:
            want = oracle.fold_table(s)
            assert score == int(want[0, -1]), (k, len(s))
            assert np.array_equal(S, want), (k, len(s))
            alone_score, alone = nf.nf_fold(s, q=8, table=True)
            assert alone_score == score and np.array_equal(alone, S), (k, len(s))
        else:
            assert score == oracle.fold_score(s), (k, len(s))
            assert score == nf.nf_fold(s, q=8), (k, len(s))


_MIXED_Q_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1307_7820_amd import gen, nf
seqs = gen.batch_sequences(300, 50, 2000, (1307, 44)) + ["", "A", "GC"]
qs = sorted({nf.nf_autotune_q(len(s)) for s in seqs})
b = nf.Batch(seqs, q=0)
b.run()
got = b.scores()
bad = [k for k, s in enumerate(seqs) if int(got[k]) != oracle.fold_score(s)]
tables = 0
for k in range(0, len(seqs), 23):
    if seqs[k]:
        assert np.array_equal(b.table(k), oracle.fold_table(seqs[k])), k
        tables += 1
alone = [k for k in range(0, len(seqs), 17) if int(got[k]) != nf.nf_fold(seqs[k], q=nf.nf_autotune_q(len(seqs[k])))]
dbs = b.structures()
sbad = [k for k in range(0, len(seqs), 29) if dbs[k] != oracle.structure(seqs[k])]
print(json.dumps({"qs": qs, "bad": bad, "alone_bad": alone, "tables": tables, "structure_bad": sbad}))
"""


def test_batch_takes_the_tuned_q_of_each_length_bucket(tmp_path):
    """nf_batch_create(q = 0): each fold takes the q tuned for its length bucket,
    the folds of each q run as one packed wavefront, and every score, table and
    structure still equals the oracle's and the fold run alone.  The tune file is
    read once per process, so the batch runs in a child process of its own."""
    import json
    import os
    import subprocess
    import sys
    tune = tmp_path / "tune.txt"
    tune.write_text("0 5\n1 6\n2 8\n3 4\n")  # n < 256: q 5, < 512: 6, < 1024: 8, < 2048: 4
    env = dict(os.environ, NF_AUTOTUNE_CACHE=str(tune))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    print("mixed-q batch child", flush=True)
    out = subprocess.run([sys.executable, "-u", "-c", _MIXED_Q_CHILD, root], env=env, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-3000:]
    res = json.loads(out.stdout.strip().splitlines()[-1])
    assert res["qs"] == [4, 5, 6, 8], res
    assert res["bad"] == [] and res["alone_bad"] == [] and res["structure_bad"] == [], res
    assert res["tables"] >= 10
