"""The allocation-free entry point (nf_fold_dev_noalloc), called through the
C ABI, against the existing entry point nf_fold_dev on the same device codes:
scores and full tables bit-exact, calls in a row with the later ones smaller
(each call reuses the static scratch the one before it filled), and no
device memory taken from torch's allocator (the library's hook) by the call.
"""

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen

pytestmark = pytest.mark.gpu


def _fold_both(nf, L, torch, n, q, seed):
    s = gen.iid_sequence(n, [1307, 60, seed])
    stream = torch.cuda.current_stream()
    codes = torch.from_numpy(nf.nf_encode(s)).cuda()
    a_score = torch.zeros(1, dtype=torch.int32, device="cuda")
    a_S = torch.zeros(max(1, n * n), dtype=torch.int16, device="cuda")
    nf.nf_fold_dev(codes, n, q, a_score, a_S if n else None, stream)
    b_score = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    b_S = torch.full((max(1, n * n),), -7, dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    print("noalloc: n=%d q=%d" % (n, q), flush=True)
    rc = L.nf_fold_dev_noalloc(codes.data_ptr(), n, q, b_score.data_ptr(), b_S.data_ptr() if n else None,
                               stream.cuda_stream)
    assert rc == 0, nf.last_error()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before  # nothing taken through the hook
    assert int(a_score.item()) == int(b_score.item()), (n, q)
    if n:  # with n = 0 there is no table, and neither call writes the placeholder
        assert torch.equal(a_S, b_S), (n, q)
    return s, int(b_score.item()), b_S


def test_noalloc_equals_fold_dev_on_calls_in_a_row():
    import torch
    from paper_1307_7820_amd import nf
    L = nf.load()
    nf.nf_init(0)
    # the largest fold that fits at q = 8, then smaller ones over the same scratch
    for n, q, seed in ((3519, 8, 1), (1000, 8, 2), (2000, 5, 3), (777, 0, 4), (130, 3, 5), (2, 8, 6), (0, 8, 7)):
        s, score, S = _fold_both(nf, L, torch, n, q, seed)
        if 0 < n <= 1000:
            want = oracle.fold_table(s)
            assert score == int(want[0, -1])
            assert np.array_equal(S.cpu().numpy().reshape(n, n), want.astype(np.int16))


def test_noalloc_refuses_a_fold_beyond_its_scratch():
    import torch
    from paper_1307_7820_amd import nf
    L = nf.load()
    codes = torch.zeros(3520, dtype=torch.uint8, device="cuda")
    rc = L.nf_fold_dev_noalloc(codes.data_ptr(), 3520, 8, None, None, None)
    assert rc == nf.NF_E_NOMEM
    # a call that fits still runs after the refusal
    s, score, _ = _fold_both(nf, L, torch, 500, 8, 8)
    assert score == oracle.fold_score(s)
