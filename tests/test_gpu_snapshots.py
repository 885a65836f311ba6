"""GPU: scalar-flux snapshots (eq. photondensity, trapezoid rule) of the
forward states from rte_forward_ex, as in the laboratory simulation of Sec. 5
(Fig. 6), against the scalar flux of the oracle's own states; chunked sources;
the laboratory workload at full size (smooth, bounded, the light moving into
the medium) and its last snapshot against the library's own final state."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import physics
from oracle.solver import Oracle

from test_gpu_parity import TOL32, TOL64, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    R.lib()
    return R


@pytest.fixture(scope="module")
def lab_small():
    spec, steps = W.lab_flux(24, 8)
    _, _, states = Oracle(spec).forward(keep_states=True)
    return spec, steps, states


@pytest.mark.parametrize("dtype,tol", [(torch.float64, TOL64), (torch.float32, TOL32)])
def test_lab_snapshots_match_oracle(rte, lab_small, dtype, tol):
    spec, steps, states = lab_small
    levels = [0] + steps + [steps[0]]  # the initial state and a repeated level
    say("lab snapshots 25x25 M8 K%d" % spec.K, dtype, levels)
    phi, _ = rte.Plan(spec, dtype).flux_snapshots(spec.mu_a, spec.mu_s, levels)
    phi = phi.cpu().numpy()
    assert phi.shape == (1, len(levels), spec.Ny + 1, spec.Nx + 1)
    assert not phi[0, 0].any()
    for k, n in enumerate(levels[1:], 1):
        assert rel(phi[0, k], physics.scalar_flux(states[0][n])) < tol, (k, n)


@pytest.mark.parametrize("chunk", [0, 1])
def test_snapshots_two_sources(rte, chunk):
    beams = [W.beam_at(0.5, 0.0, 0, 1, 0, 1, sigma_t=2.0, t0=6.0, sigma_x=0.2),
             W.beam_at(1.0, 0.5, 0, 1, 0, 1, sigma_t=2.0, t0=6.0, sigma_x=0.2, group=1)]
    spec = W.small_problem(N=20, M=12, K=60, beams=beams, seed=3)
    levels = [60, 17, 33]
    say("snapshots two sources chunk", chunk)
    _, _, states = Oracle(spec).forward(keep_states=True)
    phi, G = rte.Plan(spec, torch.float64, combo_chunk=chunk).flux_snapshots(spec.mu_a, spec.mu_s, levels)
    phi = phi.cpu().numpy()
    for q in range(2):
        for k, n in enumerate(levels):
            assert rel(phi[q, k], physics.scalar_flux(states[q][n])) < TOL64, (q, k, n)


def test_snapshot_arguments_rejected(rte):
    spec, _ = W.lab_flux(16, 8, times=(5.0,))
    pl = rte.Plan(spec, torch.float64)
    for bad in ([-1], [spec.K + 1]):
        with pytest.raises(rte.RteError):
            pl.flux_snapshots(spec.mu_a, spec.mu_s, bad)


def test_lab_full_size(rte):
    """Fig. 6 setup at 201 x 201 nodes, 32 ordinates, up to 170 ps."""
    spec, steps = W.lab_flux(200, 32)
    say("lab flux 201x201 M32 K%d" % spec.K, steps)
    pl = rte.Plan(spec, torch.float64)
    phi, _ = pl.flux_snapshots(spec.mu_a, spec.mu_s, steps)
    _, uK = pl.forward_ex(spec.mu_a, spec.mu_s)
    phi = phi[0].cpu().numpy()
    assert np.isfinite(phi).all()
    # the last level is u^K: its scalar flux from the returned state
    ref = (2.0 * np.pi / spec.M) * uK[0].double().sum(-1).cpu().numpy()
    assert rel(phi[-1], ref) < 1e-13
    y = np.linspace(spec.ymin, spec.ymax, spec.Ny + 1)
    cy = []
    for k in range(len(steps)):
        p = phi[k]
        assert p.min() > -2e-2 * p.max(), k  # spectral ringing stays small
        w = np.clip(p, 0, None).sum(1)
        cy.append(float((w * y).sum() / w.sum()))
    say("lab flux centroid y", cy, "peak", [float(p.max()) for p in phi])
    assert cy[0] < cy[1] < cy[2]
