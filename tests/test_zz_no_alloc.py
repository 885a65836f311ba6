"""GPU: rte_forward_noalloc (no workspace argument, static device scratch)
against rte_forward with a workspace, through the C ABI: bit-identical G and
u^K on two calls in a row, the second with a smaller problem, and the size
limit reported as an error."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_2202_09421_amd import rte
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib = rte.lib()
    lib.rte_forward_noalloc.argtypes = [ctypes.c_void_p] * 6
    lib.rte_forward_noalloc.restype = ctypes.c_int
    return lib


def _pair(L, spec, dtype):
    from paper_2202_09421_amd import rte
    plan = rte.Plan(spec, dtype)
    a = torch.tensor(spec.mu_a, device="cuda", dtype=dtype)
    b = torch.tensor(spec.mu_s, device="cuda", dtype=dtype)
    G_ref, u_ref = plan.forward(a, b, want_u_final=True)
    G = torch.full_like(G_ref, float("nan"))
    u = torch.full_like(u_ref, float("nan"))
    rc = L.rte_forward_noalloc(plan._h, a.data_ptr(), b.data_ptr(), G.data_ptr(), u.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    assert rc == 0, L.rte_last_error().decode()
    torch.cuda.synchronize()
    return plan, (G_ref, u_ref), (G, u)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_noalloc_forward_equals_workspace_forward(L, dtype):
    big = W.small_problem(N=40, M=16, K=30, seed=3, n_in=1.4)
    small = W.small_problem(N=17, M=8, K=45, seed=4, Ny=12)
    for spec in (big, small):   # the second call reuses the scratch with a smaller input
        print("noalloc", dtype, spec.Nx, spec.Ny, spec.M, spec.K, flush=True)
        plan, (G_ref, u_ref), (G, u) = _pair(L, spec, dtype)
        assert torch.equal(G, G_ref) and torch.equal(u, u_ref)
        plan.close()


def test_noalloc_leaves_a_saved_forward_valid(L):
    from paper_2202_09421_amd import rte
    spec = W.small_problem(N=16, M=8, K=20, seed=5)
    plan = rte.Plan(spec, torch.float64)
    a = torch.tensor(spec.mu_a, device="cuda")
    b = torch.tensor(spec.mu_s, device="cuda")
    G0 = plan.forward(a, b, save_states=True)
    gbar = torch.ones_like(G0)
    da0, db0 = plan.adjoint(gbar, a, b)
    plan.forward(a, b, save_states=True)
    G = torch.empty_like(G0)
    assert L.rte_forward_noalloc(plan._h, a.data_ptr(), b.data_ptr(), G.data_ptr(), None,
                                 torch.cuda.current_stream().cuda_stream) == 0
    da1, db1 = plan.adjoint(gbar, a, b)
    assert torch.equal(G, G0) and torch.equal(da1, da0) and torch.equal(db1, db0)


def test_noalloc_rejects_problems_beyond_the_scratch(L):
    from paper_2202_09421_amd import rte
    spec = W.config(1)    # 257 x 257 x 32 FP64: its forward needs more than the static scratch
    plan = rte.Plan(spec, torch.float64)
    a = torch.tensor(spec.mu_a, device="cuda")
    G = torch.empty((1, plan.Nd, spec.K), dtype=torch.float64, device="cuda")
    rc = L.rte_forward_noalloc(plan._h, a.data_ptr(), a.data_ptr(), G.data_ptr(), None,
                               torch.cuda.current_stream().cuda_stream)
    assert rc == rte.RTE_ENOMEM and "static scratch" in L.rte_last_error().decode()
