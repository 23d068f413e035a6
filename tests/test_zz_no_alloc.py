"""The allocation-free explicit apply (sc_apply_noalloc) against sc_apply.

Both run the same kernels in the same summation order; the allocation-free
entry point keeps the partial sums in the library's fixed per-GPU array and
runs the batch in chunks of whole subdomains.  Its output must equal
sc_apply's bit for bit, on two calls in a row, the second on a smaller plan
(the array keeps the first call's contents)."""
import numpy as np
import pytest

import scgen

P = pytest.importorskip("paper_2509_21037_amd")
pytestmark = pytest.mark.gpu


def _plan(subs, precision):
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    plan = P.Plan(subs, precision=precision)
    plan.factor()
    plan.assemble()
    return plan


def _compare(plan, seed):
    import torch
    n = plan.dual_total
    g = torch.Generator(device="cpu").manual_seed(seed)
    p = (torch.rand(n, generator=g, dtype=torch.float64) * 2 - 1).cuda()
    q_ref = torch.full_like(p, np.nan)
    q_new = torch.full_like(p, np.nan)
    plan.apply(p, q_ref)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    plan.apply_noalloc(p, q_new)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    assert not torch.isnan(q_new).any()
    assert torch.equal(q_new, q_ref)
    return q_new


def test_noalloc_apply_matches_apply_on_two_calls_in_a_row():
    # 1024 heat subdomains: 28 stored tiles each, 28672 in all, so the fixed
    # array (16384 tiles) takes the batch in two chunks
    big = _plan(scgen.config_subdomains(2), "fp64")
    small = _plan(scgen.config_subdomains(3, count=3), "mixed")
    try:
        _compare(big, 1)
        _compare(small, 2)          # second call, smaller input
        _compare(big, 3)            # and back: nothing stale from the last call
    finally:
        big.destroy()
        small.destroy()


def test_noalloc_apply_checks_its_arguments_like_apply():
    import torch
    plan = _plan(scgen.config_subdomains(1), "fp64")
    try:
        p = torch.rand(plan.dual_total, dtype=torch.float64, device="cuda")
        with pytest.raises(P.ScasmError):
            plan.apply_noalloc(p, p)                 # aliasing
        with pytest.raises(P.ScasmError):
            plan.apply_noalloc(p.float(), torch.zeros_like(p))   # wrong dtype, rejected before the call
    finally:
        plan.destroy()
