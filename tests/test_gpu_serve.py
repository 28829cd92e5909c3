"""GPU tests of the serving engine (nf_submit / nf_poll / nf_wait).

Continuous batching must not change any result: every fold served in a mix
equals the same fold run alone and the CPU oracle, bit for bit.
"""

import time

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


def _drain(nf, tickets, want_table=None, timeout_s=120):
    """Poll until every ticket completes; returns {ticket: (score, table)}."""
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, n in tickets.items():
            if t in out:
                continue
            wt = bool(want_table and want_table.get(t))
            done, score, S = nf.nf_poll(t, n, wt)
            if done:
                out[t] = (score, S)
        assert time.time() - t0 < timeout_s, "serving did not finish"
        time.sleep(0.0005)
    return out


def test_mix_equals_alone_and_oracle(nf):
    nf.nf_serve_config(0, 64, 0)
    trace = gen.serving_trace(60, 0.0, seed=(201, 0), short=(50, 400), long=(1200, 2600), p_short=0.75)
    seqs = [s for _, s in trace] + ["", "A", "GC", "ACGU" * 20]
    tickets, want = {}, {}
    for k, s in enumerate(seqs):
        t = nf.nf_submit(s, q=8, want_table=(k % 5 == 0))
        tickets[t] = len(s)
        want[t] = (k % 5 == 0)
    res = _drain(nf, tickets, want)
    for (t, n), s in zip(tickets.items(), seqs):
        score, S = res[t]
        assert score == oracle.fold_score(s), n
        if want[t]:
            assert np.array_equal(S, oracle.fold_table(s)), n
        assert score == nf.nf_fold(s, q=8)  # the same fold alone
    st = nf.nf_serve_stats()
    assert st.completed == len(seqs) and st.admitted == len(seqs)


def test_budget_binds_and_results_hold(nf):
    per = nf.nf_fold_bytes(1500, 8)
    budget = int(per * 2.5) + (4 << 20)   # room for about two long folds at a time
    nf.nf_serve_config(budget, 0, 0)
    seqs = [gen.iid_sequence(1500, [202, k]) for k in range(6)] + \
           [gen.iid_sequence(int(n), [203, k]) for k, n in enumerate(np.linspace(60, 600, 20))]
    tickets = {nf.nf_submit(s, q=8): len(s) for s in seqs}
    res = _drain(nf, tickets)
    for (t, n), s in zip(tickets.items(), seqs):
        assert res[t][0] == oracle.fold_score(s)
    st = nf.nf_serve_stats()
    assert st.peak_bytes <= budget
    assert st.peak_bytes >= per  # the budget actually held long folds


def test_errors_and_timeouts(nf):
    nf.nf_serve_config(64 << 20, 4, 3)
    with pytest.raises(nf.NFError) as e:
        nf.nf_submit(gen.iid_sequence(9000, [204, 0]))       # > 64 MB budget
    assert e.value.code == nf.NF_E_NOMEM
    with pytest.raises(nf.NFError) as e:
        nf.nf_submit("ACGT")
    assert e.value.code == nf.NF_E_INVAL
    with pytest.raises(nf.NFError) as e:
        nf.nf_poll(987654321)
    assert e.value.code == nf.NF_E_NOTFOUND
    s = gen.iid_sequence(3000, [204, 1])
    t = nf.nf_submit(s)
    # queue of 3: at most a few more fit before NF_E_BUSY
    extra, busy = [], False
    for k in range(40):
        try:
            extra.append(nf.nf_submit(gen.iid_sequence(3000, [205, k])))
        except nf.NFError as err:
            assert err.code == nf.NF_E_BUSY
            busy = True
            break
    assert busy
    score = nf.nf_wait(t, 60000)
    assert score == oracle.fold_score(s)
    with pytest.raises(nf.NFError) as e:     # released on completion
        nf.nf_poll(t)
    assert e.value.code == nf.NF_E_NOTFOUND
    for x in extra:
        nf.nf_wait(x, 60000)


def test_wait_timeout_then_complete(nf):
    nf.nf_serve_config(0, 0, 0)
    s = gen.iid_sequence(8000, [206, 0])
    t = nf.nf_submit(s)
    with pytest.raises(nf.NFError) as e:
        nf.nf_wait(t, 0)
    assert e.value.code == nf.NF_E_TIMEOUT
    assert nf.nf_wait(t, 120000) == oracle.fold_score(s)


def test_shutdown_aborts_or_completes(nf):
    nf.nf_serve_config(0, 8, 0)
    seqs = [gen.iid_sequence(2500, [207, k]) for k in range(12)]
    tickets = [nf.nf_submit(s) for s in seqs]
    nf.nf_shutdown()
    for t, s in zip(tickets, seqs):
        try:
            done, score, _ = nf.nf_poll(t)
            assert done and score == oracle.fold_score(s)
        except nf.NFError as err:
            assert err.code in (nf.NF_E_ABORTED, nf.NF_E_NOTFOUND)


def test_structures_in_a_mix(nf):
    # NF_WANT_STRUCTURE: the engine traces each fold back on the device when it
    # finishes; the structure equals the oracle's and the single-fold path's,
    # with and without the table, while other folds are in flight
    from pins import check_structure
    nf.nf_serve_config(0, 32, 0)
    trace = gen.serving_trace(40, 0.0, seed=(204, 0), short=(50, 400), long=(1200, 2600), p_short=0.75)
    seqs = [s for _, s in trace] + ["", "A", "GGGAAACCC"]
    sub = []
    for k, s in enumerate(seqs):
        wt, ws = (k % 3 == 0), (k % 3 != 2)
        sub.append((nf.nf_submit(s, q=8, want_table=wt, want_structure=ws), s, wt, ws))
    for t, s, wt, ws in sub:
        done, score, S, db = nf.nf_poll_ex(t, 120000, len(s), wt, ws)
        assert done and score == oracle.fold_score(s), len(s)
        if wt:
            assert np.array_equal(S, oracle.fold_table(s)), len(s)
        if ws:
            assert db == oracle.structure(s), len(s)
            check_structure(s, db, score)
            if s:
                assert db == nf.nf_fold_structure(s, q=8)[1], len(s)
        else:
            assert db is None
    with pytest.raises(nf.NFError) as e:
        load = nf.load()
        rc = load.nf_submit(b"ACGU", 4, 8, 4)  # unknown flag
        nf._check(rc)
    assert e.value.code == nf.NF_E_INVAL


@pytest.mark.parametrize("mode", ["fused", "staged", None])
def test_step_forms_equal_oracle(nf, mode):
    # A step runs fused (one launch per q holding its finishes and the next
    # diagonals' between work) or staged (two streams); NF_MODE, read when the
    # engine starts, forces one, and without it every step is fused.  Mixed q
    # puts several q groups into one step.
    import os
    old = os.environ.get("NF_MODE")
    if mode is None:
        os.environ.pop("NF_MODE", None)
    else:
        os.environ["NF_MODE"] = mode
    try:
        nf.nf_serve_config(0, 64, 0)
        trace = gen.serving_trace(48, 0.0, seed=(207, 0), short=(50, 400), long=(1500, 3000), p_short=0.7)
        seqs = [s for _, s in trace] + ["", "GC"]
        tickets, opts = {}, {}
        for k, s in enumerate(seqs):
            q = 5 if k % 3 == 0 else 8
            wt, ws = k % 4 == 0, k % 4 == 1
            t = nf.nf_submit(s, q=q, want_table=wt, want_structure=ws)
            tickets[t] = s
            opts[t] = (wt, ws)
        for t, s in tickets.items():
            wt, ws = opts[t]
            done, score, S, db = nf.nf_poll_ex(t, 120000, len(s), wt, ws)
            assert done and score == oracle.fold_score(s), len(s)
            if wt:
                assert np.array_equal(S, oracle.fold_table(s)), len(s)
            if ws:
                assert db == oracle.structure(s), len(s)
        st = nf.nf_serve_stats()
        assert st.completed == len(seqs)
        if mode == "staged":
            assert st.steps_fused == 0
        else:
            assert st.steps_fused == st.steps
    finally:
        nf.nf_shutdown()
        if old is None:
            os.environ.pop("NF_MODE", None)
        else:
            os.environ["NF_MODE"] = old
