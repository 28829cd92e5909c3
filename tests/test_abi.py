"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nf.h")


def _declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(nf_[A-Za-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1307_7820_amd import nf
    return nf.load()


def test_header_and_binding_agree():
    from paper_1307_7820_amd import nf
    assert sorted(nf.EXPORTS) == _declared_functions()


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    hooks = _declared_functions(os.path.join(ROOT, "include", "nf_test.h"))
    assert set(hooks) == {"nf_test_schedule", "nf_test_set_perturb", "nf_test_packed_state"}
    for name in hooks:
        assert hasattr(lib, name), name


def test_rejects_bad_input_without_device(lib):
    from paper_1307_7820_amd import nf
    # validation happens before any device call
    assert lib.nf_fold(b"ACGT", 4, 0, None) == nf.NF_E_INVAL
    assert "0x54" in nf.last_error()
    assert lib.nf_fold(b"ACGU", 4, 10, None) == nf.NF_E_INVAL
    assert lib.nf_fold(b"ACGU", -1, 0, None) == nf.NF_E_INVAL
    buf = ctypes.create_string_buffer(8)
    assert lib.nf_fold_structure(b"ACGU", 4, 0, None) == nf.NF_E_INVAL  # no output buffer
    assert lib.nf_fold_structure(b"ACGX", 4, 0, buf) == nf.NF_E_INVAL
    assert lib.nf_fold_structure(b"ACGU", 4, 10, buf) == nf.NF_E_INVAL
    assert buf.raw == b"\0" * 8  # nothing written on error
    assert lib.nf_fold(b"A", nf.NF_MAX_N + 1, 0, None) == nf.NF_E_TOOLONG
    assert lib.nf_precompute_R(0) == nf.NF_E_INVAL
    assert lib.nf_precompute_R(10) == nf.NF_E_INVAL
    buf = (ctypes.c_uint8 * 4)()
    assert lib.nf_copy_R(3, ctypes.addressof(buf), 4) == nf.NF_E_INVAL  # needs 16 bytes


def test_fold_bytes_is_host_arithmetic(lib):
    from paper_1307_7820_amd import nf
    b8 = nf.nf_fold_bytes(16000, 8)
    # dense int16 table of (NT*64)^2 cells dominates: about 516 MB at n = 16000,
    # plus 2 KB of column words and 2 KB of row words per tile (about 130 MB)
    # and the double-buffered accumulators (about 8 MB)
    assert 640e6 < b8 < 700e6
    assert nf.nf_fold_bytes(100, 8) < nf.nf_fold_bytes(1000, 8)
    assert nf.nf_fold_bytes(-1, 8) == 0


def _check_schedule(lib, nts, target):
    arr = (ctypes.c_int * len(nts))(*nts)
    msg = ctypes.create_string_buffer(256)
    rc = lib.nf_test_schedule(arr, len(nts), target, msg, 256)
    assert rc == 0, (nts[:8], target, msg.value.decode())


def test_schedule_invariants_single_folds(lib):
    # one fold of NT tiles per side (n + 1 <= 64 NT), chunk targets from one
    # chunk per tile-pair up to whole tiles
    for nt in [1, 2, 3, 4, 5, 6, 9, 17, 40, 94, 251]:
        for target in [1, 7, 64, 1024, 1 << 20]:
            _check_schedule(lib, [nt], target)


def test_schedule_invariants_batches(lib):
    import numpy as np
    rng = np.random.default_rng([601])
    for t in range(30):
        count = int(rng.integers(1, 60))
        nts = [int(x) for x in rng.integers(1, 40, size=count)]
        _check_schedule(lib, nts, int(rng.choice([1, 5, 100, 1024])))
    # the 4096-fold workload's tile counts (n log-uniform in [50, 2000], 64-post tiles)
    from paper_1307_7820_amd import gen
    nts = [(len(s) + 1 + 63) // 64 for s in gen.workload_batch4096()]
    _check_schedule(lib, nts, 1024)


def test_schedule_invariants_hold_in_perturbed_order(lib):
    # the race-detection hook shuffles every step's items; the schedule's
    # invariants (each tile once, each group tile once, slots disjoint) must
    # not depend on the order
    import numpy as np
    rng = np.random.default_rng([602])
    try:
        for seed in (1, 7, 12345):
            assert lib.nf_test_set_perturb(seed) == 0
            for nt in [1, 4, 5, 9, 40, 94]:
                for target in [1, 64, 1024]:
                    _check_schedule(lib, [nt], target)
            for t in range(5):
                nts = [int(x) for x in rng.integers(1, 40, size=int(rng.integers(2, 50)))]
                _check_schedule(lib, nts, int(rng.choice([5, 100, 1024])))
    finally:
        lib.nf_test_set_perturb(0)


def test_packed_state_hook_rejects_bad_input(lib):
    from paper_1307_7820_amd import nf
    nt = ctypes.c_int(-1)
    buf = (ctypes.c_uint32 * 8)()
    assert lib.nf_test_packed_state(b"ACGU", 4, 0, buf, buf, ctypes.c_size_t(8), ctypes.byref(nt)) == nf.NF_E_INVAL
    assert lib.nf_test_packed_state(b"A", 1, 8, buf, buf, ctypes.c_size_t(8), ctypes.byref(nt)) == nf.NF_E_INVAL
    assert lib.nf_test_packed_state(b"ACGU", 4, 8, None, buf, ctypes.c_size_t(8), ctypes.byref(nt)) == nf.NF_E_INVAL
    # n = 100 at q = 8: 64-post tiles, NT = 2, 3 tiles of 8 x 64 words per block
    assert lib.nf_test_packed_state(b"A" * 100, 100, 8, buf, buf, ctypes.c_size_t(8), ctypes.byref(nt)) == nf.NF_E_INVAL
    assert nt.value == 2 and "1536 words" in nf.last_error()


def test_schedule_hook_rejects_bad_input(lib):
    from paper_1307_7820_amd import nf
    arr = (ctypes.c_int * 2)(3, 0)
    assert lib.nf_test_schedule(arr, 2, 1024, None, 0) == nf.NF_E_INVAL
    assert lib.nf_test_schedule(arr, 1, 0, None, 0) == nf.NF_E_INVAL


def test_serving_engine_that_failed_does_not_strand_later_requests(lib):
    # Without a device the engine thread's set-up fails: the request it holds
    # completes with NF_E_DEVICE, and a request submitted after the thread has
    # ended starts a new one (which fails the same way) instead of waiting in
    # a queue that nothing serves.
    from paper_1307_7820_amd import nf
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the failure path of a machine without a GPU")
    nf.nf_shutdown()
    try:
        nf.nf_serve_config(1 << 26)
        for _ in range(2):
            t = nf.nf_submit("GGGAAACCC")
            with pytest.raises(nf.NFError) as e:
                nf.nf_wait(t, timeout_ms=10000)
            assert e.value.code == nf.NF_E_DEVICE, str(e.value)
    finally:
        nf.nf_shutdown()


def test_serving_submit_and_shutdown_race(lib):
    # Submits from several threads while another shuts the engine down again
    # and again: every ticket handed out resolves (here, without a device, to
    # an error) and none waits forever.
    import threading
    from paper_1307_7820_amd import nf
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the failure path of a machine without a GPU")
    nf.nf_shutdown()
    nf.nf_serve_config(1 << 26)
    tickets, lock, stop = [], threading.Lock(), threading.Event()

    def submitter():
        while not stop.is_set():
            try:
                t = nf.nf_submit("GGGAAACCC")
            except nf.NFError:
                continue  # refused at submit: nothing to resolve
            with lock:
                tickets.append(t)

    def stopper():
        for _ in range(50):
            nf.nf_shutdown()
            try:
                nf.nf_serve_config(1 << 26)
            except nf.NFError:
                pass  # a submit restarted the engine first

    try:
        ts = [threading.Thread(target=submitter) for _ in range(3)]
        for t in ts:
            t.start()
        stopper()
        stop.set()
        for t in ts:
            t.join(30)
        assert tickets
        for t in tickets:
            with pytest.raises(nf.NFError) as e:
                nf.nf_wait(t, timeout_ms=10000)
            assert e.value.code in (nf.NF_E_DEVICE, nf.NF_E_ABORTED), str(e.value)
    finally:
        stop.set()
        nf.nf_shutdown()


def _tuning_in_subprocess(tmp_path, lines, env_extra, lengths):
    # the tune file is read once per process: ask a fresh one
    import json
    import subprocess
    import sys
    f = tmp_path / "tune.txt"
    f.write_text("".join(l + "\n" for l in lines))
    env = {k: v for k, v in os.environ.items() if k not in ("NF_BETWEEN_TARGET", "NF_STAGE_WIDE")}
    env.update(NF_AUTOTUNE_CACHE=str(f), **env_extra)
    code = ("import json,sys; sys.path.insert(0, %r); from paper_1307_7820_amd import nf; "
            "print(json.dumps([[nf.nf_autotune_q(n), nf.nf_autotune_target(n), nf.nf_autotune_target(n, 8), "
            "int(nf.nf_autotune_wide(n, 8))] for n in %r]))" % (ROOT, lengths))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_tune_file_sets_q_and_chunk_target_per_bucket(tmp_path):
    # buckets: n < 256 is 0, then one per doubling; 6000 is in bucket 5, 16000 in 6
    lines = ["5 7 256", "6 8", "2 4 0", "9 12 512", "junk", "3 5 2048 extra"]
    # [tuned q, target at that q, target at q = 8]
    # [tuned q, target at that q, target at q = 8, wide fused step at q = 8]
    got = _tuning_in_subprocess(tmp_path, lines, {}, [6000, 16000, 700, 300, 100])
    assert got[0] == [7, 256, 1024, 0]   # both columns; the target holds for q = 7 only
    assert got[1] == [8, 1024, 1024, 1]  # no target column: the default; n >= 8192 is wide
    assert got[2] == [4, 1024, 1024, 0]  # target 0: the default
    assert got[3] == [8, 1024, 1024, 0]  # q = 12 is out of range: the whole line is ignored
    assert got[4] == [8, 1024, 1024, 0]  # no line for bucket 0
    got = _tuning_in_subprocess(tmp_path, ["5 8 512"], {}, [6000])
    assert got == [[8, 512, 512, 0]]
    got = _tuning_in_subprocess(tmp_path, ["5 7 256"], {"NF_BETWEEN_TARGET": "333"}, [6000, 100])
    assert got == [[7, 333, 333, 0], [8, 333, 333, 0]]  # the environment overrides every target
    # the fourth column: the fused-step shape tuned at that q
    got = _tuning_in_subprocess(tmp_path, ["5 8 256 1", "6 8 1024 0", "7 7 1024 1"], {}, [6000, 16000, 20000])
    assert got == [[8, 256, 256, 1], [8, 1024, 1024, 0], [7, 1024, 1024, 1]]
    got = _tuning_in_subprocess(tmp_path, ["6 8 1024 0"], {"NF_STAGE_WIDE": "1"}, [16000, 100])
    assert [g[3] for g in got] == [1, 1]  # the environment overrides the choice


def test_autotune_target_rejects_bad_length(lib):
    from paper_1307_7820_amd import nf
    assert lib.nf_autotune_target(-1, 0) == nf.NF_E_INVAL
    assert lib.nf_autotune_target(nf.NF_MAX_N + 1, 0) == nf.NF_E_INVAL
    assert lib.nf_autotune_target(100, 10) == nf.NF_E_INVAL


def test_fold_dev_checks_tensor_arguments_before_the_call():
    """The binding refuses device arguments that are too small, of the wrong
    dtype, not contiguous or on the host, before the library sees them (an
    undersized buffer would otherwise be written out of bounds)."""
    import torch
    from paper_1307_7820_amd import nf
    codes = torch.zeros(10, dtype=torch.uint8)
    with pytest.raises(ValueError, match="device tensor"):
        nf.nf_fold_dev(codes, 10, 8)
    with pytest.raises(ValueError):
        nf.nf_fold_dev(torch.zeros(10, dtype=torch.uint8), -1, 8)
    # the dtype, size and layout checks read only tensor metadata
    class Fake:
        def __init__(self, dtype, numel, contiguous=True):
            self.dtype, self._n, self._c, self.is_cuda = dtype, numel, contiguous, True

        def numel(self):
            return self._n

        def is_contiguous(self):
            return self._c

        def data_ptr(self):
            raise AssertionError("the pointer must not be taken")
    with pytest.raises(ValueError, match="uint8"):
        nf.nf_fold_dev(Fake(torch.int32, 10), 10, 8)
    with pytest.raises(ValueError, match="needs 10"):
        nf.nf_fold_dev(Fake(torch.uint8, 9), 10, 8)
    with pytest.raises(ValueError, match="contiguous"):
        nf.nf_fold_dev(Fake(torch.uint8, 10, False), 10, 8)
    ok = Fake(torch.uint8, 10)
    ok.data_ptr = lambda: 0  # checked, never used: the next argument fails
    with pytest.raises(ValueError, match="d_score"):
        nf.nf_fold_dev(ok, 10, 8, d_score=Fake(torch.int64, 1))
    with pytest.raises(ValueError, match="needs 100"):
        nf.nf_fold_dev(ok, 10, 8, d_S=Fake(torch.int16, 99))
    with pytest.raises(ValueError, match="int16"):
        nf.nf_fold_dev(ok, 10, 8, d_S=Fake(torch.int32, 100))


def test_allocator_hook_and_encode_are_host_calls(lib):
    """nf_set_allocator takes both functions or neither; nf_encode maps
    Section 2's alphabet to the codes nf_fold_dev takes, and rejects anything
    else without writing."""
    import numpy as np
    from paper_1307_7820_amd import nf
    A = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)(lambda n, c: None)
    F = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)(lambda p, c: None)
    a = ctypes.cast(A, ctypes.c_void_p)
    f = ctypes.cast(F, ctypes.c_void_p)
    assert lib.nf_set_allocator(a, None, None) == nf.NF_E_INVAL
    assert lib.nf_set_allocator(None, f, None) == nf.NF_E_INVAL
    assert lib.nf_set_allocator(a, f, None) == nf.NF_OK
    assert lib.nf_set_allocator(None, None, None) == nf.NF_OK
    nf.use_torch_allocator()  # the binding's default hook goes back in
    assert list(nf.nf_encode("ACGUacgu")) == [0, 1, 2, 3, 0, 1, 2, 3]
    assert nf.nf_encode("").size == 0
    out = np.full(4, 7, dtype=np.uint8)
    assert lib.nf_encode(b"ACTG", 4, out.ctypes.data) == nf.NF_E_INVAL
    assert "base 2" in nf.last_error()
    assert list(out) == [7, 7, 7, 7]
    assert lib.nf_encode(b"A", nf.NF_MAX_N + 1, out.ctypes.data) == nf.NF_E_TOOLONG
    with pytest.raises(nf.NFError):
        nf.nf_encode("ACGN")


def test_noalloc_schedule_closed_form_and_size_limit(lib):
    """The allocation-free entry point builds its work lists on the device
    from a closed form of the single-fold schedule: the schedule hook checks
    that form against the host's builder item by item.  Folds too large for
    its static scratch are refused on the host, before any device call."""
    from paper_1307_7820_amd import nf
    msg = ctypes.create_string_buffer(256)
    for NT in list(range(1, 70)) + [120, 251, 1024]:
        for target in (1, 7, 256, 1024, 4096):
            arr = (ctypes.c_int * 1)(NT)
            rc = lib.nf_test_schedule(arr, 1, target, msg, 256)
            assert rc == 0, (NT, target, msg.value)
    rc = lib.nf_fold_dev_noalloc(1, 3520, 8, None, None, None)
    assert rc == nf.NF_E_NOMEM and "scratch" in nf.last_error()
    assert lib.nf_fold_dev_noalloc(1, 3200, 4, None, None, None) == nf.NF_E_NOMEM
    # within the limit the call gets as far as the device, which is absent here
    assert lib.nf_fold_dev_noalloc(1, 3519, 8, None, None, None) == nf.NF_E_DEVICE
    assert lib.nf_fold_dev_noalloc(None, 10, 8, None, None, None) == nf.NF_E_INVAL
    assert lib.nf_fold_dev_noalloc(1, 10, 10, None, None, None) == nf.NF_E_INVAL
