"""GPU: the outer inverse loop driven by the library's gradient follows the
same L-BFGS-B iterates as the loop driven by the FP64 oracle's gradient
(same tiny phantom, three iterations): the same number of objective
evaluations, and iterates that agree to 1e-6 (the gradients differ at their
rounding floor, ~1e-11 here, and the quasi-Newton steps amplify that by the
conditioning of the misfit; observed 2.4e-8).  A wrong gradient moves the
iterates at O(1)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.solver import Oracle
from paper_2202_09421_amd.inverse import plan_objective, reconstruct

from test_gpu_parity import rel, say

pytestmark = pytest.mark.gpu


def test_inverse_iterates_match_oracle_driven_loop():
    from paper_2202_09421_amd import rte
    spec = W.small_problem(N=16, M=8, K=300, seed=32, n_in=1.4, g=0.8, a0=0.2, b0=5.0,
                           beams=[W.beam_at(0.5, 0.0, 0, 1.0, 0, 1.0, sigma_t=5.0, t0=15.0, sigma_x=0.2, group=0),
                                  W.beam_at(1.0, 0.5, 0, 1.0, 0, 1.0, sigma_t=5.0, t0=15.0, sigma_x=0.2, group=1)])
    X, Y = np.meshgrid(np.linspace(0, 1, 17), np.linspace(0, 1, 17))
    a_true = 0.2 + 0.4 * np.exp(-((X - 0.5) ** 2 + (Y - 0.4) ** 2) / 0.02)
    spec = spec.with_(mu_a=a_true, mu_s=np.full_like(a_true, 5.0))
    o = Oracle(spec)
    Gm = o.forward()[0]

    def oracle_fn(a):
        J, ga, _, _ = o.gradient(Gm, mu_a=a)
        return J, ga

    plan = rte.Plan(spec, torch.float64)
    a0 = np.full_like(a_true, 0.2)
    a_o, h_o = reconstruct(oracle_fn, a0, 0.2, 1.0, max_iter=3, a_true=a_true, dx=spec.dx, dy=spec.dy)
    a_g, h_g = reconstruct(plan_objective(plan, spec.mu_s, Gm), a0, 0.2, 1.0, max_iter=3, a_true=a_true,
                           dx=spec.dx, dy=spec.dy)
    say("iterations", len(h_o) - 1, len(h_g) - 1, "final E %.4f %.4f" % (h_o[-1]["E"], h_g[-1]["E"]),
        "iterate rel diff %.2e" % rel(a_g, a_o))
    assert [h["evals"] for h in h_o] == [h["evals"] for h in h_g]
    assert rel(a_g, a_o) < 1e-6
    # misfits on the scale the optimiser sees (J / J0)
    for x, y in zip(h_o, h_g):
        assert abs(x["J"] - y["J"]) <= 1e-8 * h_o[0]["J"]
