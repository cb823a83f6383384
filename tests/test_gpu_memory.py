"""Device memory of a context comes from the caller's allocator (PyTorch's
caching allocator through the binding) and goes back to it on destroy."""
import pytest

from synth import c2_dirichlet_varmu

pytestmark = pytest.mark.gpu


def _inverse_entries(nb):
    # symmetric tile layout: TR (TR + 1) / 2 tiles of 16 x 16, diagonal ones
    # storing 40 of their 64 lane blocks of 4 entries
    tr = (nb + 15) // 16
    return tr * 40 * 4 + tr * (tr - 1) // 2 * 64 * 4


def test_context_storage_is_owned_by_torch():
    import torch
    from paper_1911_05888_amd import Context, V_FP32, V_FP64, IR
    print("[memory] torch-owned context storage", flush=True)
    prob = c2_dirichlet_varmu(n=64, p=3)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = Context(prob, vprec=V_FP32, build_precisions=1 << V_FP64)
    grown = torch.cuda.memory_allocated() - base
    # at least the finest level's block inverses in FP32 and FP64
    need = prob.n_elements * _inverse_entries(prob.nb) * (4 + 8)
    assert grown >= need, (grown, need)
    b = ctx.assemble_rhs(prob.rhs_source())
    x = torch.zeros_like(b)
    st, info = ctx.solve(b, x, tol=1e-10, maxit=40, outer=IR)
    assert st == 0
    ctx.close()
    del b, x
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_library_allocation_leaves_torch_untouched():
    import torch
    from paper_1911_05888_amd import Context, V_FP32, IR
    prob = c2_dirichlet_varmu(n=32, p=3)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = Context(prob, vprec=V_FP32, torch_memory=False)
    assert torch.cuda.memory_allocated() == base
    b = ctx.assemble_rhs(prob.rhs_source())
    x = torch.zeros_like(b)
    st, info = ctx.solve(b, x, tol=1e-10, maxit=40, outer=IR)
    assert st == 0
    ctx.close()
