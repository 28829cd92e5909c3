"""Benchmark: Four-Russians Nussinov fill on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

A step is one complete fill of the n = 6000 iid uniform sequence (the
workload the headline GCUPS figure is quoted on) with codes already resident
in device memory: every kernel of the wavefront plus the score write.  The
timed region is K back-to-back steps on torch's current stream, bracketed by
torch.cuda.synchronize() and HIP events.

GCUPS = n(n+1)/2 table cells / fill time / 1e9 (R is built once, before the
timed region; no host transfers inside it).

Unless --q is given, q (4..8) and then the between-group chunks per step are
chosen first by nf_autotune, outside the timed region; config records both.

Printed beside the headline (one JSON line on stdout; progress on stderr):
  roofline      dominant kernel (by time) measured with per-launch HIP events
  cpu_baseline  the CPU oracle timed on this host on the same sequence
  extra         n = 16000 fold, 4096-sequence batch vs looped single folds,
                and the serving engine under a Poisson trace
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: int32 VALU lane-ops/s
OPS_PER_LOOKUP = 3.0                          # Eq. 3 lookup: form the R index, add the two bases and R, max
OPS_PER_TERM = 2.0                            # add + max of one Eq. 1 term
# algorithmic HBM bytes of a lookup when the packed words (int16 base + 8-bit
# difference vector, one per row and one per column of a group) are reused
# over a 64 x 64-cell tile: 2 x 3 bytes per 64 lookups
HBM_BYTES_PER_LOOKUP = 6.0 / 64
TUNE_REPS = 5                                 # folds per candidate when the headline q and chunk target are tuned
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def splits(n: int) -> float:
    """Split evaluations of plain Eq. 1 over the whole table, (n-1)n(n+1)/6:
    the inner-loop count of the plain recurrence, a method-independent rate."""
    return (n - 1) * n * (n + 1) / 6.0


def cells(n: int) -> float:
    return n * (n + 1) / 2.0


def time_fold(nf, torch, seq: str, q: int, steps: int, warmup: int):
    n = len(seq)
    codes = torch.from_numpy(nf.encode(seq)).cuda()
    d_score = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        nf.nf_fold_dev(codes, n, q, d_score, None, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        nf.nf_fold_dev(codes, n, q, d_score, None, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    return ms, wall, int(d_score.item()), codes


WORKLOAD_NAMES = {6000: "n6000", 16000: "n16000"}


def kernels_source_hash() -> str:
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1307_7820_amd", "csrc", "nf_kernels.hip")
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_bytes(kernel: str, q: int, n: int, target: int, wide: int):
    """HBM bytes per launch of `kernel`, from the committed rocprofv3 counter
    summary profiles/<kernel>_q<q>_<workload>_pmc.txt: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch, separate runs), each scaled by what the same
    counter reads for a plain device copy of known size.  The summary holds
    one `traffic:` line per launch configuration measured; the one taken at
    `target` between-group chunks per step and step shape `wide` (split
    chunks write by atomic max, so the chunks change the bytes) is used.
    None when there is no summary or no such line, or when the kernel source
    has changed since the counters were taken (its hash is in the line)."""
    wl = WORKLOAD_NAMES.get(n)
    if wl is None:
        return None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "%s_q%d_%s_pmc.txt" % (kernel, q, wl))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if not line.startswith("traffic:"):
                continue
            vals = dict(kv.partition("=")[::2] for kv in line.split()[1:])
            try:
                if vals.get("kernels_sha256") != kernels_source_hash():
                    continue
                if int(vals.get("target", "0")) != target or int(vals.get("wide", "0")) != int(wide):
                    continue
                return 1024.0 * (float(vals["fetch_kib"]) * float(vals["fetch_scale"]) +
                                 float(vals["write_kib"]) * float(vals["write_scale"]))
            except (KeyError, ValueError):
                continue
    return None


def lds_ceiling(nf, q: int):
    """Measured LDS 1-byte gather rates over a table of R's size for q:
    offsets uniform over the table, and one wave-uniform row of R with a
    random column per lane (the pattern of the between-group lookups)."""
    table = max(64, 1 << (2 * (q - 1)))
    row = 1 << (q - 1)
    uniform = nf.nf_lds_gather_rate(table, 0)
    rowwise = nf.nf_lds_gather_rate(table, row if table % row == 0 and row <= table else 0)
    return {"table_bytes": table, "row_bytes": row, "uniform_gathers_per_s": uniform, "row_gathers_per_s": rowwise}


def roofline_times(lookups: float, terms: float, cells_out: float, seconds: float, lds_rate: float):
    """t* = max(t_VALU, t_LDS, t_HBM) for the given algorithmic work, and the
    roofline object with the binding unit's achieved and peak rates (so that
    frac = achieved / peak = t* / t)."""
    t_valu = (OPS_PER_LOOKUP * lookups + OPS_PER_TERM * terms) / PEAK_VALU_LANE_OPS
    t_lds = lookups / lds_rate
    hbm_bytes = HBM_BYTES_PER_LOOKUP * lookups + 2.0 * cells_out
    t_hbm = hbm_bytes / PEAK_HBM
    t_star = max(t_valu, t_lds, t_hbm)
    if t_star == t_valu:
        out = {"bound": "alu", "achieved": (OPS_PER_LOOKUP * lookups + OPS_PER_TERM * terms) / seconds / 1e12,
               "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "TOP/s"}
    elif t_star == t_lds:
        out = {"bound": "lds", "achieved": lookups / seconds / 1e9, "peak": lds_rate / 1e9, "unit": "Ggathers/s"}
    else:
        out = {"bound": "hbm", "achieved": hbm_bytes / seconds / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["t_valu_us"], out["t_lds_us"], out["t_hbm_us"], out["t_us"] = (1e6 * t_valu, 1e6 * t_lds, 1e6 * t_hbm,
                                                                      1e6 * seconds)
    out["algorithmic_hbm_bytes"] = hbm_bytes
    return out


def roofline(nf, codes, n, q, lds, reps=3):
    """Roofline of the kernel that takes most of the fill's device time.

    Algorithmic work per launch, from the work lists (nf_profile_fold):
    3 VALU lane-ops per Eq. 3 lookup and 2 per Eq. 1 term evaluated one by
    one, one LDS byte gather per lookup, and 6/64 HBM bytes per lookup plus
    2 bytes per table cell written.  Duration = the kernel's own start and
    end, recorded into HIP events by its dispatch on the launching stream.
    The LDS rate is the measured row-pattern gather ceiling."""
    prof = nf.nf_profile_fold(codes, n, q, reps)
    target = nf.nf_autotune_target(n, q)  # the chunks per step the profiled plan was built with
    ks = [i for i in range(len(nf.KERNEL_NAMES)) if prof.launches[i] > 0]
    k = max(ks, key=lambda i: prof.ms[i])
    name = nf.KERNEL_NAMES[k]
    per_launch_s = prof.ms[k] / 1e3 / prof.launches[k]
    L = prof.lookups[k] / prof.launches[k]
    X = prof.splits[k] / prof.launches[k]
    C = prof.cells[k] / prof.launches[k]
    r = roofline_times(L, X, C, per_launch_s, lds["row_gathers_per_s"])
    traffic = traffic_bytes(name, q, n, target, prof.wide)
    out = {"kernel": name, "launches_per_fold": prof.launches[k] // reps,
           "avg_launch_us": 1e6 * per_launch_s,
           "per_kernel_ms_per_fold": {nf.KERNEL_NAMES[i]: prof.ms[i] / reps for i in ks},
           **r,
           "lookups_per_launch": L, "terms_per_launch": X, "cells_per_launch": C,
           "glookups_per_s": prof.lookups[k] / (prof.ms[k] / 1e3) / 1e9,
           "traffic": traffic,
           "hbm_achieved_gbs": traffic / per_launch_s / 1e9 if traffic else None,
           "hbm_frac": traffic / per_launch_s / PEAK_HBM if traffic else None,
           "q": prof.q, "tile": prof.tile, "between_chunks_per_step": target, "wide_fused_step": bool(prof.wide),
           "fold": {"lookups": sum(prof.lookups[i] for i in ks) / reps,
                    "terms": sum(prof.splits[i] for i in ks) / reps}}
    return out


def fold_work(n: int, q: int):
    """Algorithmic work of one fill, counted as the kernels run it (the same
    counts nf_profile_fold reports per launch, summed): Eq. 3 lookups, Eq. 1
    terms evaluated one by one, and table cells written."""
    G = 64 // q
    T = G * q
    NT = -(-(n + 1) // T)

    def valid(B):
        return max(0, min(T, n + 1 - B * T))
    lookups = terms = cells_out = 0.0
    for B in range(NT):
        v = valid(B)
        # main-diagonal tile: cell (i, i+t) has t-1 split points and a pairing term
        terms += sum((v - t) * t for t in range(1, v))
        cells_out += v * (v + 1) / 2
        if B == 0:
            continue
        between = (B - 3) * (B - 2) / 2 if B >= 4 else 0          # sum over d = 4..B of d - 3
        ends = 2 * B - 3 if B >= 2 else 0                         # sum over d = 1..B of min(d - 1, 2)
        lookups += (between + ends) * G * T * v
        own_rows = v * 8 * 28 if 8 % q == 0 else v * T * (T - 1) / 2
        block = v * 8 * 28 * (8 // q) if 8 % q == 0 else 0
        lookups += B * block
        terms += B * (T * v * (v - 1) / 2 + own_rows + T * v)
        cells_out += B * T * v
    return lookups, terms, cells_out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(seq: str, gen, budget_s: float):
    """The CPU oracle (plain Eq. 1, OpenMP over the cells of a diagonal) on
    this host, as it stands.  Headline value: whole n = 6000 folds on all the
    threads OpenMP gives it.  Beside it: one thread (a bounded sample, the
    first 3000 bases, scaled to n = 6000 by the split count, since its time
    is proportional to (n-1)n(n+1)/6), and the batch workload (512 of the 4096
    sequences, one thread each on as many workers as the oracle's threads)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    threads = oracle.threads_used()
    n = len(seq)
    t0 = time.perf_counter()
    reps = 0
    score = None
    while True:
        score = oracle.fold_score(seq)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / reps * (reps + 1) > 2 * budget_s:
            break
    per = el / reps
    sub = seq[:3000]
    t0 = time.perf_counter()
    oracle.fold_score(sub, nthreads=1)
    one = time.perf_counter() - t0
    one_scaled = one * splits(n) / splits(len(sub))
    seqs = gen.workload_batch4096()[::8]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda x: oracle.fold_score(x, nthreads=1), seqs))
    bt = time.perf_counter() - t0
    out = {"value": cells(n) / per / 1e9, "unit": "GCUPS", "cores": threads, "kind": "oracle",
           "sample": "%d full fold(s) of the n=%d sequence on %d OpenMP threads, %.2f s each" % (reps, n, threads, per),
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "single_thread": {"value": cells(n) / one_scaled / 1e9, "unit": "GCUPS", "cores": 1,
                             "sample": "one fold of the first %d bases, %.2f s, scaled by split count to n=%d (%.1f s)"
                                       % (len(sub), one, n, one_scaled)},
           "batch4096": {"value": len(seqs) / bt, "unit": "folds/s", "cores": threads,
                         "sample": "%d of the 4096 batch sequences (every 8th), one thread each on %d workers, %.2f s"
                                   % (len(seqs), threads, bt)}}
    return out, score


def extra_n16000(nf, torch, gen, steps, lds):
    """The n = 16000 fold with q, the chunk target and the fused-step shape
    chosen by the autotuner for its length (tuned before the timed region)."""
    seq = gen.workload_n16000()
    n = len(seq)
    t0 = time.perf_counter()
    q = nf.nf_autotune(n, 4, 8, 2)
    tune_s = time.perf_counter() - t0
    ms, wall, score, codes = time_fold(nf, torch, seq, q, steps, 1)
    t = ms / 1e3 / steps
    r = roofline(nf, codes, n, q, lds, reps=1)
    return {"n": 16000, "q": q, "between_chunks_per_step": nf.nf_autotune_target(n, q),
            "wide_fused_step": nf.nf_autotune_wide(n, q), "autotune_s": tune_s,
            "ms_per_fold": t * 1e3, "gcups": cells(16000) / t / 1e9,
            "split_equivalent_gsps": splits(16000) / t / 1e9,
            "glookups_per_s": r.get("glookups_per_s"), "score": score, "roofline": r}


def extra_q_sweep(nf, torch, gen, steps=3):
    """The n=6000 fold at every q.  At q = 1 a group holds a single split
    point and R is the 1x1 zero table, so the same wavefront evaluates the
    splits of Eq. 1 one by one: the plain recurrence, the ablation of the
    Four-Russians lookup."""
    seq = gen.workload_n6000()
    out = {}
    for q in range(1, 9):
        ms, wall, score, codes = time_fold(nf, torch, seq, q, steps, 1)
        t = ms / 1e3 / steps
        out["q%d" % q] = {"ms_per_fold": t * 1e3, "gcups": cells(len(seq)) / t / 1e9, "score": score}
    out["fr_speedup_q8_over_q1"] = out["q1"]["ms_per_fold"] / out["q8"]["ms_per_fold"]
    # n = 16000, where the between-group lookups dominate: q = 1 against q = 8
    seq = gen.workload_n16000()
    big = {}
    for q in (1, 8):
        ms, wall, score, codes = time_fold(nf, torch, seq, q, 1, 1)
        big["q%d" % q] = {"ms_per_fold": ms, "gcups": cells(len(seq)) / (ms / 1e3) / 1e9, "score": score}
    big["fr_speedup_q8_over_q1"] = big["q1"]["ms_per_fold"] / big["q8"]["ms_per_fold"]
    out["n16000"] = big
    return out


def extra_plain_ablation(nf, torch, gen):
    """n=16000 on staged steps, the between-group work by the lookup kernel
    and by the plain-recurrence kernel (NF_BETWEEN=plain, packed 16-bit adds
    and maxima, no R); per-kernel times from nf_profile_fold."""
    seq = gen.workload_n16000()
    n = len(seq)
    out = {}
    for label, env in (("lookup", {"NF_MODE": "staged"}), ("plain", {"NF_MODE": "staged", "NF_BETWEEN": "plain"})):
        old = {k: os.environ.get(k) for k in env}
        os.environ.update(env)
        try:
            ms, wall, score, codes = time_fold(nf, torch, seq, 8, 1, 1)
            prof = nf.nf_profile_fold(codes, n, 8, 1)
            out[label] = {"ms_per_fold": ms, "score": score,
                          "between_ms": prof.ms[2], "tile_ms": prof.ms[1], "between_launches": prof.launches[2]}
        finally:
            for k, v in old.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
    out["between_speedup_lookup_over_plain"] = out["plain"]["between_ms"] / out["lookup"]["between_ms"]
    return out


def extra_structure(nf, gen, reps=3):
    """Traceback through D* (nf_fold_structure) beside the fill alone
    (nf_fold); both are synchronous host calls on the same sequence, so the
    difference is the traceback kernel plus the n-byte structure copy."""
    out = {}
    for name, seq in (("n6000", gen.workload_n6000()), ("n16000", gen.workload_n16000())):
        score, db = nf.nf_fold_structure(seq)
        nf.nf_fold(seq)
        t0 = time.perf_counter()
        for _ in range(reps):
            nf.nf_fold(seq)
        t1 = time.perf_counter()
        for _ in range(reps):
            nf.nf_fold_structure(seq)
        t2 = time.perf_counter()
        fold_ms, both_ms = (t1 - t0) / reps * 1e3, (t2 - t1) / reps * 1e3
        out[name] = {"fold_ms": fold_ms, "fold_structure_ms": both_ms, "traceback_ms": both_ms - fold_ms,
                     "pairs": score, "unpaired": db.count(".")}
    return out


def extra_batch(nf, torch, gen, lds):
    """The 4096-sequence batch: one prepared batch (q tuned per length bucket,
    one packed wavefront per q, captured as HIP graphs) against the same 4096
    folds run one by one with the single-fold call at the same q (device
    codes, every plan made and captured before the timed loop), both timed
    over all 4096 folds; and the batch at a fixed q = 8."""
    seqs = gen.workload_batch4096()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3

    def time_batch(b):
        b.run(stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            b.run(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    # q for each length bucket of the batch (n < 256, < 512, < 1024, < 2048),
    # tuned at one length inside each bucket before the timed region
    t0 = time.perf_counter()
    bucket_q = {str(m): nf.nf_autotune(m, 4, 8, 3) for m in (181, 362, 724, 1448)}
    tune_s = time.perf_counter() - t0
    b8 = nf.Batch(seqs, q=8)
    ms_q8 = time_batch(b8)
    scores_q8 = b8.scores()
    b8.close()
    t0 = time.perf_counter()
    b = nf.Batch(seqs, q=0)
    prep = time.perf_counter() - t0
    ms = time_batch(b)
    scores = b.scores()
    # structures of all 4096 folds (nf_batch_structures: one traceback
    # workgroup per fold, host call including the copies)
    b.structures()
    t0 = time.perf_counter()
    dbs = b.structures()
    structures_ms = (time.perf_counter() - t0) * 1e3
    b.close()
    # the same folds looped one by one
    cds = [torch.from_numpy(nf.encode(s)).cuda() for s in seqs]
    d_scores = torch.zeros(len(seqs), dtype=torch.int32, device="cuda")
    for i, c in enumerate(cds):  # makes and captures every single-fold plan
        nf.nf_fold_dev(c, len(seqs[i]), 0, d_scores[i:i + 1], None, stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for i, c in enumerate(cds):
        nf.nf_fold_dev(c, len(seqs[i]), 0, d_scores[i:i + 1], None, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    looped_same = bool(torch.equal(d_scores.cpu(), torch.from_numpy(scores)))
    tot_cells = sum(cells(len(s)) for s in seqs)
    work = [fold_work(len(s), nf.nf_autotune_q(len(s))) for s in seqs]
    roof = roofline_times(sum(w[0] for w in work), sum(w[1] for w in work), sum(w[2] for w in work), ms / 1e3,
                          lds["row_gathers_per_s"])
    return {"count": len(seqs), "q": "tuned per length bucket", "bucket_q": bucket_q, "autotune_s": tune_s,
            "ms_per_batch": ms, "folds_per_s": len(seqs) / (ms / 1e3),
            "ms_per_batch_q8": ms_q8, "scores_equal_q8": bool((scores == scores_q8).all()),
            "gcups": tot_cells / (ms / 1e3) / 1e9, "prepare_s": prep,
            "looped_ms_all": loop_ms, "looped_folds_per_s": len(seqs) / (loop_ms / 1e3),
            "speedup_vs_looped": loop_ms / ms, "looped_scores_equal_batch": looped_same,
            "roofline_whole_fill": roof, "score_checksum": int(scores.sum()),
            "structures_ms": structures_ms, "structure_pairs": sum(db.count("(") for db in dbs)}


def _pct(xs, p):
    import numpy as np
    return float(np.percentile(np.asarray(xs), p)) if xs else None


def extra_serving(nf, torch, gen, count=2000, warm=200, budget=2 << 30):
    """FIFO single folds (plain) vs the continuous-batching engine (served).

    Same request sequence for both (lengths 80% U{100..500}, 20% U{2000..8000},
    iid bases): `warm` requests to warm up, then `count` measured ones.
    Saturation: every request available at t=0.  Open loop: Poisson arrivals
    at 0.8 x the plain saturation rate; latency = completion observed by the
    caller - arrival.  budget = device bytes the active folds may hold (0: 80%
    of the free device memory when the engine starts).
    """
    import threading
    import numpy as np
    trace = gen.serving_trace(count + warm, 1.0, seed=(1307, 5))
    seqs = [s for _, s in trace]
    stream = torch.cuda.current_stream()
    codes = [torch.from_numpy(nf.encode(s)).cuda() for s in seqs]
    d_score = torch.zeros(1, dtype=torch.int32, device="cuda")
    for c, s in zip(codes, seqs):  # warm every single-fold plan
        nf.nf_fold_dev(c, len(s), 8, d_score, None, stream)
    torch.cuda.synchronize()
    meas = list(range(warm, warm + count))

    def plain_one(i):
        nf.nf_fold_dev(codes[i], len(seqs[i]), 8, d_score, None, stream)
        torch.cuda.synchronize()

    t0 = time.perf_counter()
    for i in meas:
        plain_one(i)
    plain_T = time.perf_counter() - t0
    mu_plain = count / plain_T

    nf.nf_shutdown()
    torch.cuda.empty_cache()  # a budget of 0 reads the device's free memory
    nf.nf_serve_config(budget, 256, 0)

    def served_run(arrivals):
        tick = {}
        done_t = {}
        t_start = time.perf_counter()

        def submitter():
            for k, i in enumerate(meas):
                if arrivals is not None:
                    dt = t_start + arrivals[k] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                tick[k] = nf.nf_submit(seqs[i], 8)

        th = threading.Thread(target=submitter)
        th.start()
        outstanding = set()
        seen = 0
        while len(done_t) < len(meas):
            while seen < len(tick):
                outstanding.add(seen)
                seen += 1
            for k in list(outstanding):
                done, _, _ = nf.nf_poll(tick[k])
                if done:
                    done_t[k] = time.perf_counter() - t_start
                    outstanding.discard(k)
            time.sleep(0.0001)
        th.join()
        return done_t, time.perf_counter() - t_start

    # warm the engine: a few folds, then one untimed saturation pass (its
    # staging buffers grow to the size a full queue needs)
    ws = [nf.nf_submit(seqs[i], 8) for i in range(warm)]
    for t in ws:
        nf.nf_wait(t, 600000)
    served_run(None)
    # two short spin kernels bracket the timed saturation pass in a kernel
    # trace (bench.py --summarize busy takes the device-busy fraction between
    # them)
    torch.cuda._sleep(1000)
    done_t, served_T = served_run(None)
    torch.cuda._sleep(1000)
    mu_served = count / served_T

    lam = 0.8 * mu_plain
    rng = np.random.default_rng([1307, 6])
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=count))
    # plain, open loop: one fold at a time in arrival order
    lat_plain = []
    t_start = time.perf_counter()
    for k, i in enumerate(meas):
        dt = t_start + arrivals[k] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        plain_one(i)
        lat_plain.append(time.perf_counter() - t_start - arrivals[k])
    # served, open loop
    done_t, _ = served_run(arrivals)
    lat_served = [done_t[k] - arrivals[k] for k in range(count)]
    st = nf.nf_serve_stats()
    nf.nf_shutdown()
    torch.cuda.empty_cache()
    return {
        "requests": count, "warmup_requests": warm, "budget_bytes": int(st.budget_bytes),
        "mean_n": float(np.mean([len(seqs[i]) for i in meas])),
        "saturation_folds_per_s": {"plain_fifo": mu_plain, "served": mu_served},
        "open_loop_rate_per_s": lam,
        "latency_ms_plain": {"p50": 1e3 * _pct(lat_plain, 50), "p99": 1e3 * _pct(lat_plain, 99)},
        "latency_ms_served": {"p50": 1e3 * _pct(lat_served, 50), "p99": 1e3 * _pct(lat_served, 99)},
        "served_over_plain_throughput": mu_served / mu_plain,
        "engine_steps": int(st.steps), "engine_steps_fused": int(st.steps_fused), "peak_bytes": int(st.peak_bytes),
    }


def extra_serial(gen):
    """The paper's serial CPU algorithms (Section 3; libnf_serial.so) on this
    host, one thread, at two of the lengths of the paper's serial table, with
    the plain recurrence they are compared against; and the two-vector method
    on every thread (diagonal order).  Context for the paper's ratios."""
    from paper_1307_7820_amd import serial
    out = {"cpu_model": cpu_model()}
    for n in (2000, 4000):
        seq = gen.iid_sequence(n, [1307, 2])
        row = {}
        for label, q, variant, threads in (("plain", 1, "plain", 1), ("two_vector_q8", 8, "two_vector", 1),
                                           ("partial_memo_q8", 8, "partial_memo", 1),
                                           ("full_memo_q8", 8, "full_memo", 1), ("fg_q3", 3, "fg", 1),
                                           ("two_vector_q8_all_threads", 8, "two_vector", os.cpu_count() or 1)):
            t0 = time.perf_counter()
            score, st = serial.nf_serial_fold(seq, q, variant, threads)
            row[label] = {"s": time.perf_counter() - t0, "score": score, "threads": threads,
                          "lookups": st.lookups, "r_entries": st.r_entries}
        for k in list(row):
            if k != "plain":
                row[k]["speedup_over_plain"] = row["plain"]["s"] / row[k]["s"]
        out["n%d" % n] = row
    return out


def run_only(args, torch, gen, nf):
    """One workload, warm-up then K runs, for rocprofv3 kernel traces and counters."""
    if args.only == "copy":
        # plain device-to-device copy of 1 GiB: calibrates FETCH_SIZE / WRITE_SIZE
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        for _ in range(args.warmup + args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"only": "copy", "bytes_per_copy": x.numel(), "copies": args.warmup + args.steps}))
        return
    nf.nf_init(0)
    if args.only == "ldsgather":
        print(json.dumps({"only": "ldsgather", **{"q%d" % q: lds_ceiling(nf, q) for q in (4, 6, 8, 9)}}))
        return
    if args.only == "serving":
        # the serving extra alone (plain FIFO, saturation, open loop)
        print(json.dumps({"only": "serving", **extra_serving(nf, torch, gen)}))
        return
    if args.only == "batch":
        seqs = gen.workload_batch4096()
        b = nf.Batch(seqs, q=8)
        for _ in range(args.warmup + args.steps):
            b.run(torch.cuda.current_stream())
        torch.cuda.synchronize()
        print(json.dumps({"only": "batch", "count": len(seqs), "checksum": int(b.scores().sum())}))
        return
    if args.only in ("structure6000", "structure16000"):
        # fill + traceback through D* (nf_fold_structure), K times
        seq = gen.workload_n6000() if args.only == "structure6000" else gen.workload_n16000()
        for _ in range(args.warmup + args.steps):
            score, db = nf.nf_fold_structure(seq, q=args.q if args.q else 8)
        print(json.dumps({"only": args.only, "n": len(seq), "pairs": score}))
        return
    if args.only == "plain16000":
        # n=16000 on staged steps with the plain-recurrence between kernel
        os.environ["NF_MODE"] = "staged"
        os.environ["NF_BETWEEN"] = "plain"
        seq = gen.workload_n16000()
    else:
        seq = gen.workload_n6000() if args.only == "n6000" else gen.workload_n16000()
    q = args.q if args.q else 8
    ms, wall, score, _ = time_fold(nf, torch, seq, q, args.steps, args.warmup)
    print(json.dumps({"only": args.only, "n": len(seq), "q": q,
                      "between_chunks_per_step": nf.nf_autotune_target(len(seq), q), "ms_per_fold": ms / args.steps,
                      "gcups": cells(len(seq)) * args.steps / (ms / 1e3) / 1e9, "score": score}))


# ---------------------------------------------------------------- summaries
# Summaries of rocprofv3 result databases (SQLite, *_results.db), for the
# text files under profiles/: per-kernel durations, per-dispatch counter
# means and the device-busy fraction of the library's kernels.

_KERNEL_KEYS = ("k_stage<", "k_diag<", "k_between_plain<", "k_between<", "k_tile<", "k_traceback_many",
                "k_traceback", "k_scores", "k_copy_codes", "k_precompute_R", "k_expand", "k_lds_gather",
                "k_single_items", "k_zero", "k_delay")


def _short_name(name):
    for key in _KERNEL_KEYS:
        if key in name:
            i = name.index(key)
            return name[i:name.find(">", i) + 1] if key.endswith("<") else key
    return name[:40]


def summarize_trace(db):
    """Per-kernel call count, total / mean / min / max duration (us) and share."""
    import collections
    import sqlite3
    agg = collections.defaultdict(list)
    for name, dur in sqlite3.connect(db).execute("select name, duration from kernels"):
        agg[_short_name(name)].append(dur / 1e3)
    tot = sum(sum(v) for v in agg.values())
    return ["%-22s calls=%6d total_us=%12.1f avg_us=%9.2f min_us=%9.2f max_us=%9.2f pct=%5.1f"
            % (k, len(v), sum(v), sum(v) / len(v), min(v), max(v), 100 * sum(v) / tot)
            for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))]


def summarize_pmc(db, kernel):
    """Per-dispatch mean of every counter, over the dispatches of kernels whose name holds `kernel`."""
    import collections
    import sqlite3
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    q = "select kernel_name, counter_name, dispatch_id, value from counters_collection"
    for k, c, d, v in sqlite3.connect(db).execute(q):
        if kernel in k:
            per[c][d] += v
    return {c: (len(v), sum(v.values()) / len(v)) for c, v in per.items()}


def summarize_busy(db):
    """Fraction of time at least one of the library's kernels runs: over the
    span of all of them, and over each window between consecutive
    torch.cuda._sleep marker kernels."""
    import sqlite3
    rows = list(sqlite3.connect(db).execute("select name, start, end from kernels order by start"))
    lib = sorted((s, e) for n, s, e in rows if _short_name(n).startswith("k_") and "k_delay" not in n)
    marks = [s for n, s, e in rows if "sleep" in n.lower() or "spin" in n.lower()]

    def busy(lo, hi):
        tot, cs, ce = 0, None, None
        for s, e in lib:
            s, e = max(s, lo), min(e, hi)
            if e <= s:
                continue
            if cs is None or s > ce:
                if cs is not None:
                    tot += ce - cs
                cs, ce = s, e
            else:
                ce = max(ce, e)
        if cs is not None:
            tot += ce - cs
        return tot / max(1, hi - lo), (hi - lo) / 1e9

    out = {"span": busy(lib[0][0], lib[-1][1]) if lib else (0.0, 0.0)}
    for k, (a, b) in enumerate(zip(marks, marks[1:])):
        out["window%d" % k] = busy(a, b)
    return out


def run_summarize(args):
    kind, db = args.summarize[0], args.summarize[1]
    if kind == "trace":
        print("\n".join(summarize_trace(db)))
    elif kind == "pmc":
        kernel = args.summarize[2] if len(args.summarize) > 2 else "k_"
        for c, (n, m) in sorted(summarize_pmc(db, kernel).items()):
            print("%-28s dispatches=%5d mean=%16.1f" % (c, n, m))
    elif kind == "busy":
        for k, (b, span) in summarize_busy(db).items():
            print("%-10s device busy %.3f of %.3f s" % (k, b, span))
    else:
        sys.exit("--summarize trace|pmc|busy DB [KERNEL]")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--q", type=int, default=0)
    ap.add_argument("--cpu-budget-s", type=float, default=10.0)
    ap.add_argument("--quick", action="store_true", help="headline only (no extra workloads)")
    ap.add_argument("--only", choices=["n6000", "n16000", "batch", "copy", "structure6000", "structure16000",
                                       "plain16000", "serving", "ldsgather"],
                    help="run one workload K times and print a short line (for profilers)")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="trace|pmc|busy DB [KERNEL]: summarize a rocprofv3 result database and exit")
    args = ap.parse_args()
    if args.summarize:
        run_summarize(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a single fold is a "
              "latency-bound wavefront; batches and serving shard by fold). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1307_7820_amd import gen, nf

    if args.only:
        run_only(args, torch, gen, nf)
        return
    nf.nf_init(0)
    seq = gen.workload_n6000()
    n = len(seq)
    if args.q:
        q = args.q
    else:
        # q in 4..8, then the chunk target at that q, by timing (not timed here)
        t0 = time.perf_counter()
        q = nf.nf_autotune(n, 4, 8, TUNE_REPS)
        log("bench: autotune n=%d: q=%d, chunk target %d (%.2f s)"
            % (n, q, nf.nf_autotune_target(n), time.perf_counter() - t0))
    target = nf.nf_autotune_target(n, q)
    log("bench: n=%d q=%d target=%d warmup=%d steps=%d" % (n, q, target, args.warmup, args.steps))
    ms, wall, score, codes = time_fold(nf, torch, seq, q, args.steps, args.warmup)
    ms_per = ms / args.steps
    value = cells(n) * args.steps / (ms / 1e3) / 1e9
    log("bench: %.3f ms/fold, %.2f GCUPS, score %d" % (ms_per, value, score))
    lds = lds_ceiling(nf, q)
    log("bench: lds gather ceiling %s" % json.dumps(lds))
    roof = roofline(nf, codes, n, q, lds)
    log("bench: roofline %s" % json.dumps(roof))
    fw = fold_work(n, q)
    if abs(fw[0] - roof["fold"]["lookups"]) > 1e-6 * fw[0] or abs(fw[1] - roof["fold"]["terms"]) > 1e-6 * fw[1]:
        log("bench: work count mismatch: %s vs %s" % (fw, roof["fold"]))
        sys.exit(1)
    fold_roof = roofline_times(fw[0], fw[1], fw[2], ms_per / 1e3, lds["row_gathers_per_s"])
    cpu, cpu_score = cpu_baseline(seq, gen, args.cpu_budget_s)
    log("bench: cpu baseline %s" % json.dumps(cpu))
    if cpu_score != score:
        log("bench: SCORE MISMATCH gpu %d vs oracle %d" % (score, cpu_score))
        sys.exit(1)
    extra = {}
    if not args.quick:
        try:
            extra["n16000"] = extra_n16000(nf, torch, gen, 3, lds)
            log("bench: n16000 %s" % json.dumps(extra["n16000"]))
        except Exception as e:  # reported, never hidden
            extra["n16000"] = {"error": repr(e)}
        try:
            extra["batch4096"] = extra_batch(nf, torch, gen, lds)
            log("bench: batch %s" % json.dumps(extra["batch4096"]))
        except Exception as e:
            extra["batch4096"] = {"error": repr(e)}
        try:
            extra["q_sweep_n6000"] = extra_q_sweep(nf, torch, gen)
            log("bench: q sweep %s" % json.dumps(extra["q_sweep_n6000"]))
        except Exception as e:
            extra["q_sweep_n6000"] = {"error": repr(e)}
        try:
            extra["plain_ablation_n16000"] = extra_plain_ablation(nf, torch, gen)
            log("bench: plain ablation %s" % json.dumps(extra["plain_ablation_n16000"]))
        except Exception as e:
            extra["plain_ablation_n16000"] = {"error": repr(e)}
        try:
            extra["structure"] = extra_structure(nf, gen)
            log("bench: structure %s" % json.dumps(extra["structure"]))
        except Exception as e:
            extra["structure"] = {"error": repr(e)}
        for label, budget in (("serving_2GiB", 2 << 30), ("serving_free_hbm", 0)):
            try:
                extra[label] = extra_serving(nf, torch, gen, budget=budget)
                log("bench: %s %s" % (label, json.dumps(extra[label])))
            except Exception as e:
                extra[label] = {"error": repr(e)}
        try:
            extra["serial_cpu"] = extra_serial(gen)
            log("bench: serial %s" % json.dumps(extra["serial_cpu"]))
        except Exception as e:
            extra["serial_cpu"] = {"error": repr(e)}
    line = {
        "metric": "Nussinov GCUPS at n=6000/16000; batched folds/s + p99 latency vs plain",
        "value": value, "unit": "GCUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "split_equivalent_gsps": splits(n) / (ms_per / 1e3) / 1e9,
        "dtype": "int16", "data": "synthetic",
        "config": {"workload": "single iid uniform ACGU sequence, n=6000, two-vector Four-Russians fill",
                   "n": n, "q": q, "between_chunks_per_step": target, "autotuned": not args.q,
                   "tile": roof.get("tile"), "score": score},
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": roof,
        "roofline_whole_fold": fold_roof,
        "lds_gather_ceiling": lds,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
