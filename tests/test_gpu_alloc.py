"""The allocator hook (nf_set_allocator): with the binding's default hook,
torch's caching allocator supplies the library's device memory, and the
results are the oracle's either way."""

import numpy as np
import pytest

import oracle
from paper_1307_7820_amd import gen

pytestmark = pytest.mark.gpu


def test_fold_under_torch_allocator_matches_oracle_and_uses_torch_memory():
    import torch
    from paper_1307_7820_amd import nf
    nf.nf_shutdown()
    nf.use_torch_allocator()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s = gen.iid_sequence(3001, [1307, 41])
    score, T = nf.nf_fold(s, q=8, table=True)
    want = oracle.fold_table(s)
    assert score == int(want[0, -1]) and np.array_equal(T, want)
    held = torch.cuda.memory_allocated() - before
    # the cached workspace: at least the dense int16 table of 3008^2 posts
    assert held >= 3008 * 3008 * 2, held
    nf.nf_shutdown()  # every buffer goes back to torch
    assert torch.cuda.memory_allocated() == before


def test_hipmalloc_when_the_hook_is_removed():
    import torch
    from paper_1307_7820_amd import nf
    nf.nf_shutdown()
    nf.nf_set_allocator(None, None)
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        s = gen.iid_sequence(1500, [1307, 42])
        score, T = nf.nf_fold(s, q=6, table=True)
        assert np.array_equal(T, oracle.fold_table(s))
        assert torch.cuda.memory_allocated() == before
    finally:
        nf.nf_shutdown()
        nf.use_torch_allocator()


def test_hook_failure_is_nomem_and_leaves_the_library_usable():
    from paper_1307_7820_amd import nf
    nf.nf_shutdown()
    nf.nf_set_allocator(lambda nbytes: 0, lambda ptr: None)
    try:
        with pytest.raises(nf.NFError) as e:
            nf.nf_fold(gen.iid_sequence(700, [1307, 43]), q=8)
        assert e.value.code == nf.NF_E_NOMEM
    finally:
        nf.use_torch_allocator()
    s = gen.iid_sequence(700, [1307, 43])
    assert nf.nf_fold(s, q=8) == oracle.fold_score(s)
    nf.nf_shutdown()
