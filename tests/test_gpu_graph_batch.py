"""GPU: graph-recorded gradients and uneven batches in one graph launch.

A graph replays exactly the kernels of the eager path in the same order, so
its results must equal the eager ones bit for bit.  Each replay is checked,
with eager work on other plans and a synchronisation between replays."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    R.lib()
    return R


def _gm(spec, seed):
    rng = np.random.default_rng(seed)
    return torch.tensor(1e-3 * rng.standard_normal((spec.Nq, len(spec.detectors), spec.K)), device="cuda")


def _eager(rte, spec, ckpt=0):
    plan = rte.Plan(spec, torch.float64, ckpt_every=ckpt)
    J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, _gm(spec, 1))
    torch.cuda.synchronize()
    return [x.cpu().numpy().copy() for x in (J, ga, gb, G)]


def test_graph_replays_equal_eager(rte):
    spec = W.small_problem(N=24, M=16, K=40, seed=3, n_in=1.4)
    ref = _eager(rte, spec)
    other = W.small_problem(N=16, M=8, K=20, seed=4)
    plan = rte.Plan(spec, torch.float64)
    plan.set_graph(True)
    a = torch.tensor(spec.mu_a, device="cuda")
    b = torch.tensor(spec.mu_s, device="cuda")
    gm = _gm(spec, 1)
    for rep in range(4):
        say("graph replay", rep)
        J, ga, gb, G = plan.gradient(a, b, gm)
        torch.cuda.synchronize()
        got = [x.cpu().numpy() for x in (J, ga, gb, G)]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), rep
        _eager(rte, other)          # unrelated eager work between replays
        torch.zeros(1 << 20, device="cuda").add_(1.0)
        torch.cuda.synchronize()


def test_uneven_batch_one_launch_equals_individual(rte):
    specs = [
        W.small_problem(N=24, M=16, K=40, seed=3, n_in=1.4),
        W.small_problem(N=12, M=8, K=25, seed=5),
        W.small_problem(N=20, M=12, K=60, seed=6, Ny=14, g=0.7),
        W.small_problem(N=64, M=32, K=15, seed=7, n_in=1.4, g=0.9),
    ]
    ckpts = [0, 0, 7, 0]
    refs = [_eager(rte, s, c) for s, c in zip(specs, ckpts)]
    plans = [rte.Plan(s, torch.float64, ckpt_every=c) for s, c in zip(specs, ckpts)]
    batch = rte.Batch(plans)
    media = [(torch.tensor(s.mu_a, device="cuda"), torch.tensor(s.mu_s, device="cuda")) for s in specs]
    gms = [_gm(s, 1) for s in specs]
    for rep in range(3):
        say("batch launch", rep)
        J, ga, gb, G = batch.gradient(media, gms)
        torch.cuda.synchronize()
        for i, ref in enumerate(refs):
            got = [J[i].cpu().numpy(), ga[i].cpu().numpy(), gb[i].cpu().numpy(), G[i].cpu().numpy()]
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), (rep, i)
        _eager(rte, specs[1])
        torch.cuda.synchronize()


def test_graph_gradient_workload_equals_eager(rte):
    # the benchmark's configuration, graph mode vs eager
    spec = W.config(1)
    say("graph on", spec.name)
    plan = rte.Plan(spec, torch.float64)
    a = torch.full((spec.Ny + 1, spec.Nx + 1), 0.2, dtype=torch.float64, device="cuda")
    b = torch.full((spec.Ny + 1, spec.Nx + 1), 50.0, dtype=torch.float64, device="cuda")
    gm = _gm(spec, 2)
    J0, ga0, gb0, G0 = [x.clone() for x in plan.gradient(a, b, gm)]
    plan.set_graph(True)
    for rep in range(2):
        J, ga, gb, G = plan.gradient(a, b, gm)
        torch.cuda.synchronize()
        assert torch.equal(J, J0) and torch.equal(ga, ga0) and torch.equal(gb, gb0) and torch.equal(G, G0), rep


def test_batched_mss_equals_plain_solves(rte):
    # three combinations of staggered beams in one plan ("batched") against
    # one plan per combination ("plain"): the per-combination arithmetic is
    # the same, and the gradient maps are summed over the combinations in the
    # same order, so G and the gradients agree bit for bit
    import dataclasses
    L = 1.0
    beams = [W.beam_at(0.5 * L, 0.0, 0, L, 0, L, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=0),
             W.beam_at(0.5 * L, L, 0, L, 0, L, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=0, tau=3.0),
             W.beam_at(0.0, 0.4 * L, 0, L, 0, L, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=1, tau=1.0),
             W.beam_at(L, 0.7 * L, 0, L, 0, L, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=2, tau=2.0)]
    spec = W.small_problem(N=24, M=16, K=40, seed=31, n_in=1.4, beams=beams)
    plan = rte.Plan(spec, torch.float64)
    assert plan.Nq == 3
    gm = torch.tensor(1e-3 * np.random.default_rng(3).standard_normal((3, plan.Nd, spec.K)), device="cuda")
    J, ga, gb, G = [x.cpu().numpy().copy() for x in plan.gradient(spec.mu_a, spec.mu_s, gm)]
    ga_sum = gb_sum = None
    Js = 0.0
    for q in range(3):
        sq = spec.with_(beams=[dataclasses.replace(b, group=0) for b in spec.beams if b.group == q])
        pq = rte.Plan(sq, torch.float64)
        Jq, gaq, gbq, Gq = [x.cpu().numpy().copy() for x in pq.gradient(spec.mu_a, spec.mu_s, gm[q:q + 1])]
        assert np.array_equal(Gq[0], G[q]), q
        ga_sum = gaq if ga_sum is None else ga_sum + gaq
        gb_sum = gbq if gb_sum is None else gb_sum + gbq
        Js += float(Jq[0])
    assert np.array_equal(ga_sum, ga) and np.array_equal(gb_sum, gb)
    assert abs(Js - float(J[0])) <= 1e-13 * abs(Js)



def _three_combination_spec():
    L = 1.0
    beams = [W.beam_at(0.5 * L, 0.0, 0, L, 0, L, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=0),
             W.beam_at(0.5 * L, L, 0, L, 0, L, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=1, tau=3.0),
             W.beam_at(0.0, 0.4 * L, 0, L, 0, L, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=2, tau=1.0)]
    return W.small_problem(N=24, M=16, K=30, seed=33, n_in=1.4, beams=beams)


@pytest.mark.parametrize("chunk,ckpt", [(1, 0), (2, 0), (2, 7)])
def test_combination_chunks_equal_unchunked(rte, chunk, ckpt):
    # solving the sources in chunks (workspace for `chunk` sources) gives the
    # same detector traces and gradient maps bit for bit, through rte_gradient
    # and through rte_forward + rte_adjoint (which recomputes the forward of
    # the chunks not left in the workspace); J agrees to rounding
    spec = _three_combination_spec()
    gm = torch.tensor(1e-3 * np.random.default_rng(4).standard_normal((3, 4, spec.K)), device="cuda")
    ref = rte.Plan(spec, torch.float64, ckpt_every=ckpt)
    assert ref.Nq == 3
    J0, ga0, gb0, G0 = [x.cpu().numpy().copy() for x in ref.gradient(spec.mu_a, spec.mu_s, gm)]
    pl = rte.Plan(spec, torch.float64, ckpt_every=ckpt, combo_chunk=chunk)
    assert pl.workspace_bytes() < ref.workspace_bytes()
    J, ga, gb, G = [x.cpu().numpy().copy() for x in pl.gradient(spec.mu_a, spec.mu_s, gm)]
    assert np.array_equal(G, G0) and np.array_equal(ga, ga0) and np.array_equal(gb, gb0)
    assert abs(float(J[0]) - float(J0[0])) <= 1e-14 * abs(float(J0[0]))
    G2 = pl.forward(spec.mu_a, spec.mu_s, save_states=True)
    gbar = spec.dt * (G2 - gm)
    da, db = pl.adjoint(gbar)
    torch.cuda.synchronize()
    assert np.array_equal(G2.cpu().numpy(), G0)
    assert np.array_equal(da.cpu().numpy(), ga0) and np.array_equal(db.cpu().numpy(), gb0)
    # a second adjoint starts from the chunk the first one left in the workspace
    da2, db2 = pl.adjoint(gbar)
    torch.cuda.synchronize()
    assert np.array_equal(da2.cpu().numpy(), ga0)
