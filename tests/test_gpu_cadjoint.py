"""GPU: the continuous-adjoint gradient (rte_gradient_continuous) against the
oracle's continuous adjoint (oracle/cadjoint.py), through the C ABI.

The psi solve is a forward solve driven by the detector residual, so the
halves are checked separately: J and G must equal rte_gradient's bit for bit
(same forward and misfit); the gradient maps are compared with the oracle's
continuous adjoint driven by the library's own traces G, to max(1e-10,
4 x floor) in FP64 (floor: the oracle's dense-matrix path with the same
residual) and 1e-5 in FP32.  Checkpointed replay and combination chunks must
reproduce the kept-state result bit for bit."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.cadjoint import continuous_gradient
from oracle.solver import Oracle

from test_gpu_parity import CASES, TOL32, TOL64, _measured, rel, say, tol

pytestmark = pytest.mark.gpu

CADJ_CASES = [0, 1, 2, 3, 5, 7, 9, 10]   # several FFT sizes, ragged grids, M = 4..80 (1..5 row tiles)


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    R.lib()
    return R


def _spec(i):
    return W.small_problem(**CASES[i])


@pytest.mark.parametrize("i", CADJ_CASES)
def test_continuous_gradient_fp64_matches_oracle(rte, i):
    spec = _spec(i)
    say("continuous adjoint fp64", CASES[i])
    o = Oracle(spec)
    Gm = _measured(o.forward()[0], 300 + i)
    plan = rte.Plan(spec, torch.float64)
    J, ga, gb, G = plan.gradient_continuous(spec.mu_a, spec.mu_s, Gm)
    J2, _, _, G2 = plan.gradient(spec.mu_a, spec.mu_s, Gm)
    torch.cuda.synchronize()
    assert torch.equal(J, J2) and torch.equal(G, G2)
    Gl = G.cpu().numpy()
    _, ga_o, gb_o, _ = continuous_gradient(o, Gm, G_res=Gl)
    _, ga_f, gb_f, _ = continuous_gradient(Oracle(spec, dense_derivative=True), Gm, G_res=Gl)
    errs = dict(ga=rel(ga.cpu(), ga_o), gb=rel(gb.cpu(), gb_o))
    floors = dict(ga=rel(ga_f, ga_o), gb=rel(gb_f, gb_o))
    say("  errors %s floors %s" % ({k: "%.1e" % v for k, v in errs.items()}, {k: "%.1e" % v for k, v in floors.items()}))
    for k in errs:
        assert errs[k] < tol(floors[k]), (k, errs[k], floors[k])


@pytest.mark.parametrize("i", [1, 5])
def test_continuous_gradient_fp32_matches_oracle(rte, i):
    spec = _spec(i)
    o = Oracle(spec)
    Gm = _measured(o.forward()[0], 310 + i)
    plan = rte.Plan(spec, torch.float32)
    J, ga, gb, G = plan.gradient_continuous(spec.mu_a, spec.mu_s, Gm)
    torch.cuda.synchronize()
    _, ga_o, gb_o, _ = continuous_gradient(o, Gm, G_res=G.cpu().numpy())
    e = (rel(ga.cpu(), ga_o), rel(gb.cpu(), gb_o))
    say("continuous adjoint fp32", CASES[i], "errors %.1e %.1e" % e)
    assert max(e) < TOL32


def test_continuous_gradient_checkpoints_and_chunks_bitwise(rte):
    spec = W.small_problem(N=20, M=16, K=17, seed=41, n_in=1.4, g=0.9,
                           beams=[W.beam_at(0.5, 0.0, 0, 1.0, 0, 1.0, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=0),
                                  W.beam_at(0.0, 0.5, 0, 1.0, 0, 1.0, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=1)])
    rng = np.random.default_rng(7)
    Gm = 1e-6 * rng.standard_normal((2, len(spec.detectors), spec.K))
    outs = {}
    for ck, chunk in ((0, 0), (5, 0), (0, 1), (4, 1)):
        plan = rte.Plan(spec, torch.float64, ckpt_every=ck, combo_chunk=chunk)
        outs[(ck, chunk)] = [x.cpu().numpy().copy() for x in plan.gradient_continuous(spec.mu_a, spec.mu_s, Gm)]
        plan.close()
    ref = outs[(0, 0)]
    for key, got in outs.items():
        say("checkpoint/chunk", key)
        for k, (x, y) in enumerate(zip(got, ref)):
            assert np.array_equal(x, y), (key, k)


def test_continuous_vs_discrete_gradient_on_device(rte):
    # the oracle pin's problem at 25 x 25 nodes: the library reproduces the
    # discretisation gap between the two gradients that the oracle shows
    spec = W.small_problem(N=24, M=16, K=600, seed=3, n_in=1.4, g=0.8, L=1.0, dt=0.146 * 12 / 24,
                           beams=[W.beam_at(0.5, 0.0, 0, 1.0, 0, 1.0, sigma_t=5.0, t0=15.0, sigma_x=0.2)])
    spec = spec.with_(mu_a=np.full_like(spec.mu_a, 0.5), mu_s=np.full_like(spec.mu_s, 5.0))
    plan = rte.Plan(spec, torch.float64)
    G = plan.forward(spec.mu_a, spec.mu_s)
    Gm = 0.5 * G
    _, ga_d, gb_d, _ = plan.gradient(spec.mu_a, spec.mu_s, Gm)
    _, ga_c, gb_c, _ = plan.gradient_continuous(spec.mu_a, spec.mu_s, Gm)
    ea = abs(float(ga_c.sum() - ga_d.sum())) / abs(float(ga_d.sum()))
    eb = abs(float(gb_c.sum() - gb_d.sum())) / abs(float(gb_d.sum()))
    say("continuous vs discrete directional derivative (da = 1, db = 1): %.3e %.3e" % (ea, eb))
    assert 0.02 < ea < 0.1 and 0.02 < eb < 0.1
