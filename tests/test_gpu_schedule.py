"""GPU: launch schedules and the autotuner.

The four-step line kernel with one or two work units per wave and the node
passes with any number of tiles per workgroup run the same arithmetic per
element in the same order, so their results must agree bit for bit.  The
generic Stockham line kernel computes the same operator with a different
FFT factorisation: it must agree to rounding (checked against the oracle
tolerance used by the parity tests)."""
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


def _grad(rte, spec, sched=None, dtype=torch.float64):
    plan = rte.Plan(spec, dtype)
    if sched is not None:
        plan.set_schedule(sched)
    rng = np.random.default_rng(5)
    gm = torch.tensor(1e-4 * rng.standard_normal((plan.Nq, plan.Nd, spec.K)), device="cuda")
    J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, gm)
    G2, uK = plan.forward(spec.mu_a, spec.mu_s, want_u_final=True)
    torch.cuda.synchronize()
    return [x.cpu().numpy().copy() for x in (J, ga, gb, G, uK)], plan


# N = 64 (N_p = 90, four-step), M = 16 (one row tile: 1, 2 or 4 tiles per
# block) and M = 32 (two row tiles: 1, 2 or 4 tiles per block)
@pytest.mark.parametrize("M", [16, 32])
def test_schedules_bitwise_equal(rte, M):
    spec = W.small_problem(N=64, M=M, K=20, seed=21, n_in=1.4, g=0.9)
    ref, plan = _grad(rte, spec)
    say("default schedule", plan.schedule())
    for sched in ({"line_units_per_wave": 1}, {"line_units_per_wave": 2, "node_tiles_per_block": 1},
                  {"node_tiles_per_block": 2}, {"node_tiles_per_block": 4}, {"line_waves_per_unit": 2},
                  {"line_units_per_wave": 1, "line_waves_per_unit": 2},
                  {"line_units_per_wave": 1, "line_waves_per_unit": 2, "line_global_tables": 1},
                  {"line_units_per_wave": 2, "line_global_tables": 1}):
        say("schedule", sched)
        got, _ = _grad(rte, spec, sched)
        for k, (x, y) in enumerate(zip(got, ref)):
            assert np.array_equal(x, y), (sched, k)


def test_generic_line_kernel_agrees(rte):
    spec = W.small_problem(N=64, M=16, K=20, seed=22, n_in=1.4)
    ref, _ = _grad(rte, spec)
    got, _ = _grad(rte, spec, {"line_generic": 1})
    for k, (x, y) in enumerate(zip(got, ref)):
        err = np.linalg.norm(np.ravel(x - y)) / max(np.linalg.norm(np.ravel(y)), 1e-300)
        say("generic vs four-step, output %d: rel %.2e" % (k, err))
        assert err < 1e-10, (k, err)


def test_schedule_rejects_out_of_range(rte):
    spec = W.small_problem(N=16, M=32, K=4, seed=23)
    plan = rte.Plan(spec, torch.float64)
    for bad in ({"line_units_per_wave": 3}, {"line_generic": 2}, {"node_tiles_per_block": 3},
                {"node_tiles_per_block": 8}, {"line_waves_per_unit": 4}, {"line_global_tables": 2}):
        with pytest.raises(rte.RteError):
            plan.set_schedule(bad)
    big = rte.Plan(W.small_problem(N=12, M=80, K=2, seed=24), torch.float64)
    with pytest.raises(rte.RteError):
        big.set_schedule({"node_tiles_per_block": 2})
    assert big.schedule()["node_tiles_per_block"] == 1


def test_autotune_picks_admissible_schedule(rte, tmp_path):
    spec = W.small_problem(N=64, M=32, K=20, seed=25, n_in=1.4, g=0.9)
    ref, _ = _grad(rte, spec)
    plan = rte.Plan(spec, torch.float64)
    cache = str(tmp_path / "sched.json")
    chosen = plan.autotune(spec.mu_a, spec.mu_s, cache=cache)
    say("autotuned", chosen)
    assert chosen["cached"] is False
    assert chosen["line_units_per_wave"] in (1, 2) and chosen["node_tiles_per_block"] in (1, 2, 4)
    assert chosen["line_waves_per_unit"] in (1, 2)
    assert plan.schedule() == {k: chosen[k] for k in plan.schedule()}
    again = rte.Plan(spec, torch.float64).autotune(spec.mu_a, spec.mu_s, cache=cache)
    assert again["cached"] is True and {k: again[k] for k in plan.schedule()} == plan.schedule()
    got, _ = _grad(rte, spec, plan.schedule())
    for k, (x, y) in enumerate(zip(got, ref)):
        if chosen["line_generic"]:
            err = np.linalg.norm(np.ravel(x - y)) / max(np.linalg.norm(np.ravel(y)), 1e-300)
            assert err < 1e-10, (k, err)
        else:
            assert np.array_equal(x, y), k


def test_time_kernels(rte):
    spec = W.small_problem(N=64, M=32, K=10, seed=26, n_in=1.4)
    ref, plan = _grad(rte, spec)
    us = plan.time_kernels(spec.mu_a, spec.mu_s, reps=5)
    say("kernel times (us)", us)
    assert set(us) == set(rte.KERNEL_CLASSES) and all(0.0 < v < 1e5 for v in us.values())
    # the workspace was scratch for the timing: a later gradient is unaffected
    got, _ = _grad(rte, spec)
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
