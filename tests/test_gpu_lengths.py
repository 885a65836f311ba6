"""GPU: every extended FFT length N_p from 36 to 1200 against the FP64 oracle.

Each 5-smooth N_p is reached with E = 0 by a grid of n = N_p - C nodes along
x on a thin strip (10 nodes along y, 4 ordinates, 3 steps, Fresnel
boundary), so the x lines run through the line kernel the plan picks for
that length: the four-step kernel (all lengths from 45 to 1200 with a split
into two register codelets, 1125 excepted) or the generic one.

The checks separate the forward and adjoint halves: u^K to 1e-10; the
detector traces G to max(1e-10, 4 x floor) (floor: the oracle's FFT path
against its dense-matrix path); J against the oracle's misfit of the
library's own G; dJ/dmu_a and dJ/dmu_s against the oracle's adjoint driven
by the same adjoint sources dt (G - G_meas) the library used, to
max(1e-10, 4 x the same floor of the adjoint)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.solver import Oracle

from test_gpu_parity import TOL64, _measured, rel, say, tol

pytestmark = pytest.mark.gpu

FC_C = 25


def smooth5(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


LENGTHS = [n for n in range(36, 1201) if smooth5(n)]


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    R.lib()
    return R


# node counts whose extension E is large (C + E > 38: a continuation matrix
# of more than 384 entries, read from global memory by the four-step kernel)
LARGE_E = [(140, 180), (177, 216), (248, 288), (281, 320), (310, 360), (430, 480)]


@pytest.mark.parametrize("n,Np", LARGE_E)
def test_large_extension_matches_oracle(rte, n, Np):
    _check_length(rte, n, Np)


@pytest.mark.parametrize("Np", LENGTHS)
def test_line_length_matches_oracle(rte, Np):
    _check_length(rte, Np - FC_C, Np)


def _check_length(rte, n, Np):
    spec = W.small_problem(N=n - 1, M=4, K=3, Ny=9, seed=1000 + Np, n_in=1.4, g=0.8)
    o = Oracle(spec)
    od = Oracle(spec, dense_derivative=True)
    G_o, uK_o, st = o.forward(keep_states=True)
    G_d, _, st_d = od.forward(keep_states=True)
    Gm = _measured(G_o, Np)
    plan = rte.Plan(spec, torch.float64)
    assert plan.Np_x == Np
    _, uK = plan.forward(spec.mu_a, spec.mu_s, want_u_final=True)
    J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, Gm)
    torch.cuda.synchronize()
    G = G.cpu().numpy()
    src = spec.dt * (G - Gm)
    ga_o, gb_o = o.adjoint(src, st)
    ga_d, gb_d = od.adjoint(src, st_d)
    errs = dict(u=rel(uK.cpu(), uK_o), G=rel(G, G_o), J=abs(J.item() - o.misfit(G, Gm)) / o.misfit(G, Gm),
                ga=rel(ga.cpu(), ga_o), gb=rel(gb.cpu(), gb_o))
    floors = dict(G=rel(G_d, G_o), ga=rel(ga_d, ga_o), gb=rel(gb_d, gb_o))
    say("N_p %d: %s floors %s" % (Np, {k: "%.1e" % v for k, v in errs.items()},
                                  {k: "%.1e" % v for k, v in floors.items()}))
    assert errs["u"] < TOL64 and errs["J"] < TOL64
    for k in ("G", "ga", "gb"):
        assert errs[k] < tol(floors[k]), (k, errs[k], floors[k])
    plan.close()
