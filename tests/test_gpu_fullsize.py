"""GPU parity at the configured full-size plan shapes, through the whole
gradient (forward, misfit, exact adjoint; discrete eqs. AdjointProblem and
FDwin22), element by element against the FP64 oracle's stored results
(tests/golden/make_fullsize.py, which calls only the oracle):
  * bench257: the FP64 gradient workload's plan (257 x 257 nodes, 32
    ordinates, N_p = 288 x and y lines, autotuned schedule as in the
    benchmark), K = 300 with the detectors lit;
  * mss513: the batched MSS workload's plan (513 x 513 nodes, 64 ordinates,
    N_p = 540, 4 row tiles of slots), two combinations in one plan solved in
    chunks of one with checkpoints every 4 steps (segment replays), K = 15.
G, J, dJ/dmu_a and dJ/dmu_s are compared by relative L2 against their own
norms; the bar is max(1e-10, 4 x the oracle's rounding floor of that
quantity) in FP64 and 1e-5 in FP32."""
import os

import numpy as np
import pytest
import torch

from test_gpu_parity import TOL32, rel, say, tol
from tests.golden.make_fullsize import CASES, fullsize_case, path

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    return R


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", CASES)
def test_full_size_gradient_matches_oracle(rte, name, dtype):
    if not os.path.exists(path(name)):
        pytest.fail("missing oracle fixture %s: run python -m tests.golden.make_fullsize" % path(name))
    spec, _, settings = fullsize_case(name)
    ref = np.load(path(name))
    floor = dict(zip(("G", "J", "ga", "gb"), ref["floor"]))
    say("full size", name, dtype, spec.Nx + 1, spec.M, spec.Nq, spec.K, settings)
    plan = rte.Plan(spec, dtype, **settings)
    sched = plan.autotune(spec.mu_a, spec.mu_s, cache=False)
    J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, ref["Gm"])
    torch.cuda.synchronize()
    errs = dict(G=rel(G.cpu(), ref["G"]), J=abs(J.item() - float(ref["J"])) / abs(float(ref["J"])),
                ga=rel(ga.cpu(), ref["ga"]), gb=rel(gb.cpu(), ref["gb"]))
    say("  schedule", sched)
    say("  errors", {k: "%.2e (floor %.2e)" % (v, floor[k]) for k, v in errs.items()})
    say("  |G| max %.3e, |G|/|G_meas - G| %.2f" % (np.abs(ref["G"]).max(),
        np.linalg.norm(ref["G"]) / np.linalg.norm(ref["Gm"] - ref["G"])))
    for k, v in errs.items():
        bar = tol(floor[k]) if dtype == torch.float64 else TOL32
        assert v < bar, (k, v, bar)
    plan.close()
