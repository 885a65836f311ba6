"""GPU: rte_forward_ex on the manufactured-solution problem (Sec. 5) against
the oracle's manufactured-solution solve (same q, u0, start-up history and
inflow data, built by the library's helper and by the oracle independently),
then the paper's convergence check on the device: fourth order in dt and
spectral in the ordinates.  Also: with no extra data the extended forward
equals rte_forward bit for bit."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.mms import mms_forward
from oracle.solver import Oracle
from paper_2202_09421_amd.mms import manufactured_inputs

from test_gpu_parity import TOL32, TOL64, rel, say

pytestmark = pytest.mark.gpu

A, B = 0.35, 20.0


def _spec(N, M, dt, T=0.5, L=3.0, Ny=None):
    K = int(round(T / dt))
    sp = W.small_problem(N=N, M=M, K=K, L=L, g=0.0, n_in=1.0, dt=dt, heterogeneous=False, a0=A, b0=B, Ny=Ny)
    return sp.with_(n_out=1.0)


def _device(rte, sp, dtype=torch.float64):
    plan = rte.Plan(sp, dtype)
    u0, uh, src, inflow = manufactured_inputs(sp, A, B)
    _, uK = plan.forward_ex(sp.mu_a, sp.mu_s, u0=u0, u_hist=uh, source=src, inflow=inflow)
    torch.cuda.synchronize()
    return uK[0].cpu().numpy().astype(np.float64), plan


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    R.lib()
    return R


@pytest.mark.parametrize("N,M,dt,Ny", [(16, 8, 0.02, None), (24, 12, 0.01, 17), (40, 20, 0.01, None)])
def test_mms_forward_matches_oracle(rte, N, M, dt, Ny):
    sp = _spec(N, M, dt, T=0.2, Ny=Ny)
    uK, _ = _device(rte, sp)
    u_o, _ = mms_forward(Oracle(sp), A, B)
    say("mms N=%d M=%d dt=%g: u rel %.2e" % (N, M, dt, rel(uK, u_o)))
    assert rel(uK, u_o) < TOL64


def test_mms_forward_fp32(rte):
    sp = _spec(24, 12, 0.01, T=0.2)
    uK, _ = _device(rte, sp, torch.float32)
    u_o, _ = mms_forward(Oracle(sp), A, B)
    say("mms fp32: u rel %.2e" % rel(uK, u_o))
    assert rel(uK, u_o) < TOL32


def test_forward_ex_without_extras_equals_forward(rte):
    sp = W.small_problem(N=20, M=16, K=15, seed=51, n_in=1.4, g=0.9)
    plan = rte.Plan(sp, torch.float64)
    G1, u1 = plan.forward(sp.mu_a, sp.mu_s, want_u_final=True)
    G2, u2 = plan.forward_ex(sp.mu_a, sp.mu_s)
    assert torch.equal(G1, G2) and torch.equal(u1, u2)


def test_mms_convergence_on_device(rte):
    from oracle import physics
    from oracle.mms import flux_exact

    def err(N, M, dt):
        sp = _spec(N, M, dt)
        uK, _ = _device(rte, sp)
        return np.abs(physics.scalar_flux(uK) - flux_exact(Oracle(sp), sp.K * sp.dt)).max()

    et = [err(64, 32, dt) for dt in (0.04, 0.02, 0.01)]
    ea = [err(48, M, 0.002) for M in (4, 8, 12)]
    say("device time errors", ["%.3e" % e for e in et], "angular", ["%.3e" % e for e in ea])
    for e0, e1 in zip(et, et[1:]):
        assert 12.0 < e0 / e1 < 20.0
    assert ea[0] > 100 * ea[1] and ea[1] > 50 * ea[2]
