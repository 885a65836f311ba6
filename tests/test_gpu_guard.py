"""GPU: the non-finite guard (rte_plan_set_guard).  A NaN in a medium map or a
time step far beyond the stiff limit gives non-finite outputs, which the
guard reports as RTE_EUNSTABLE (without it the call returns them silently);
on a healthy problem the guard changes nothing."""
import numpy as np
import pytest
import torch

import workloads as W

from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    R.lib()
    return R


def _spec():
    return W.small_problem(N=16, M=8, K=60, seed=7)


def _unstable(rte, plan, call):
    with pytest.raises(rte.RteError) as ei:
        call()
    assert ei.value.code == rte.RTE_EUNSTABLE
    assert "non-finite" in rte.lib().rte_last_error().decode()


def test_nan_in_medium(rte):
    spec = _spec()
    a = spec.mu_a.copy()
    a[5, 7] = np.nan
    Gm = np.zeros((1, len(spec.detectors), spec.K))
    plan = rte.Plan(spec, torch.float64)
    say("guard: NaN in mu_a")
    G = plan.forward(a, spec.mu_s)
    assert not np.isfinite(G.cpu().numpy()).all()  # unguarded: returned as is
    plan.set_guard(True)
    _unstable(rte, plan, lambda: plan.forward(a, spec.mu_s))
    _unstable(rte, plan, lambda: plan.gradient(a, spec.mu_s, Gm))
    _unstable(rte, plan, lambda: plan.gradient_continuous(a, spec.mu_s, Gm))
    _unstable(rte, plan, lambda: plan.forward_ex(a, spec.mu_s))


def test_stiff_time_step(rte):
    spec = _spec().with_(K=400)
    b = np.full_like(spec.mu_s, 1.0e4)  # c dt (a + b) ~ 30, far outside AB4's real-axis interval
    plan = rte.Plan(spec, torch.float64)
    plan.set_guard(True)
    say("guard: stiff dt, c dt b = %.1f" % (spec.c * spec.dt * 1e4))
    _unstable(rte, plan, lambda: plan.forward(spec.mu_a, b))


def test_guard_keeps_healthy_results(rte):
    spec = _spec()
    Gm = np.random.default_rng(2).standard_normal((1, len(spec.detectors), spec.K)) * 1e-3
    ref = [x.cpu().numpy() for x in rte.Plan(spec, torch.float64).gradient(spec.mu_a, spec.mu_s, Gm)]
    plan = rte.Plan(spec, torch.float64)
    plan.set_guard(True)
    for graph in (False, True):
        plan.set_graph(graph)
        got = [x.cpu().numpy() for x in plan.gradient(spec.mu_a, spec.mu_s, Gm)]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), graph


def test_guard_in_a_batch(rte):
    specs = [_spec(), W.small_problem(N=20, M=8, K=40, seed=9)]
    plans = [rte.Plan(s, torch.float64) for s in specs]
    for p in plans:
        p.set_guard(True)
    gms = [np.zeros((1, len(s.detectors), s.K)) for s in specs]
    good = [(s.mu_a, s.mu_s) for s in specs]
    batch = rte.Batch(plans)
    J, _, _, _ = batch.gradient(good, gms)  # healthy: no error
    assert all(np.isfinite(j.item()) for j in J)
    bad_a = specs[1].mu_a.copy()
    bad_a[3, 4] = np.inf
    batch2 = rte.Batch(plans)
    say("guard: batch with an Inf node in the second instance")
    _unstable(rte, plans[1], lambda: batch2.gradient([good[0], (bad_a, specs[1].mu_s)], gms))
