"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bar: relative L2 <= 1e-10 in FP64 and <= 1e-5 in FP32.  The final state u^K
is held to 1e-10 outright.  The detector traces G (and J and the gradients
that derive from them) are small weighted sums of boundary values; when the
detectors see little light their relative rounding floor can exceed 1e-10.
For those quantities the tolerance is max(1e-10, 4 * floor), where floor is
the disagreement of the oracle with itself when the same FC operators are
applied through dense matrices instead of the FFT (same mathematics, another
rounding order).  Small cases span several FFT sizes, ragged grids (Nx != Ny,
the minimum 2d nodes per side), ordinate counts that leave part of an MFMA
tile empty (M = 4, 12, 20), several MSS combinations and K = 1.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle.solver import Oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    return R


def floor_forward(spec):
    """Rounding floor of (G, u^K): oracle FFT path vs oracle dense path."""
    Ga, ua, _ = Oracle(spec).forward()
    Gb, ub, _ = Oracle(spec, dense_derivative=True).forward()
    return rel(Gb, Ga), rel(ub, ua)


def floor_gradient(spec, Gm):
    """Rounding floors of (G, J, dJ/da, dJ/db): the dense-path disagreement, and
    the effect on J and the gradients of random relative perturbations of G of
    the size of G's own floor (the detector traces feed the adjoint sources)."""
    a = Oracle(spec)
    Ga, _, st = a.forward(keep_states=True)
    Ja = a.misfit(Ga, Gm)
    gaa, gba = a.adjoint(spec.dt * (Ga - Gm), st)
    Jb, gab, gbb, Gb = Oracle(spec, dense_derivative=True).gradient(Gm)
    f = dict(G=rel(Gb, Ga), J=abs(Ja - Jb) / abs(Ja), ga=rel(gab, gaa), gb=rel(gbb, gba))
    for trial in range(3):
        dG = np.random.default_rng(1000 + trial).standard_normal(Ga.shape)
        dG *= max(f["G"], 1e-16) * np.linalg.norm(Ga) / np.linalg.norm(dG)
        gap, gbp = a.adjoint(spec.dt * (Ga + dG - Gm), st)
        f["J"] = max(f["J"], abs(a.misfit(Ga + dG, Gm) - Ja) / abs(Ja))
        f["ga"] = max(f["ga"], rel(gap, gaa))
        f["gb"] = max(f["gb"], rel(gbp, gba))
    return f


def tol(floor, base=TOL64):
    return max(base, 4.0 * floor)


def _measured(G, seed):
    rng = np.random.default_rng(seed)
    return G * (1 + 0.3 * rng.standard_normal(G.shape)) + 0.05 * np.abs(G).max() * rng.standard_normal(G.shape)


CASES = [
    dict(N=12, M=8, K=30, seed=1),
    dict(N=16, M=16, K=40, seed=2, n_in=1.4),
    dict(N=20, M=12, K=25, seed=3, Ny=13, n_in=1.33),
    dict(N=9, M=4, K=20, seed=4, Ny=9),                    # 10 nodes = 2d per side
    dict(N=40, M=20, K=15, seed=5, g=0.8),
    dict(N=64, M=32, K=12, seed=6, n_in=1.4, g=0.9),
    dict(N=30, M=16, K=1, seed=7),                          # a single step
    dict(N=16, M=48, K=10, seed=8, n_in=1.4),               # 3 row tiles of 16 slots
    dict(N=14, M=64, K=8, seed=9, n_in=1.4, g=0.9),         # 4 row tiles
    dict(N=12, M=80, K=6, seed=10, n_in=1.33),              # 5 row tiles (runtime tile count)
    dict(N=64, M=16, K=10, seed=11, Ny=20, n_in=1.4),       # four-step x lines, generic y lines
    dict(N=128, M=8, K=6, seed=12, n_in=1.4),               # N_p = 160 (16 x 10 split)
    dict(N=1024, M=4, K=6, seed=13, Ny=9, n_in=1.4),        # x lines N_p = 1080 (long four-step variant)
    dict(N=9, M=8, K=6, seed=14, Ny=700, n_in=1.33),        # y lines N_p = 729 = 3^6 (generic)
    # degenerate media: isotropic scattering with an index-matched boundary
    # (no reflection), no scattering at all, no absorption in a homogeneous
    # medium
    dict(N=16, M=8, K=20, seed=15, g=0.0, n_in=1.0),
    dict(N=16, M=12, K=20, seed=16, b0=0.0, n_in=1.4),
    dict(N=16, M=8, K=20, seed=17, a0=0.0, heterogeneous=False),
]
GRAD_CASES = [0, 1, 2, 3, 4, 5, 7, 8, 9, 10, 12, 13, 14, 15, 16]


def _spec(case):
    c = dict(case)
    return W.small_problem(**c)


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_forward_fp64_matches_oracle(rte, case):
    spec = _spec(case)
    say("forward fp64", case)
    o = Oracle(spec)
    G_o, uK_o, _ = o.forward()
    plan = rte.Plan(spec, torch.float64)
    G, uK = plan.forward(spec.mu_a, spec.mu_s, want_u_final=True)
    torch.cuda.synchronize()
    fG, fu = floor_forward(spec)
    say("  G %.2e (floor %.2e)  u %.2e (floor %.2e)" % (rel(G.cpu(), G_o), fG, rel(uK.cpu(), uK_o), fu))
    assert rel(G.cpu(), G_o) < tol(fG), rel(G.cpu(), G_o)
    assert rel(uK.cpu(), uK_o) < TOL64, rel(uK.cpu(), uK_o)


@pytest.mark.parametrize("case", [CASES[i] for i in GRAD_CASES], ids=[str(i) for i in GRAD_CASES])
def test_gradient_fp64_matches_oracle(rte, case):
    spec = _spec(case)
    say("gradient fp64", case)
    o = Oracle(spec)
    Gm = _measured(o.forward()[0], 100 + case["seed"])
    J_o, ga_o, gb_o, G_o = o.gradient(Gm)
    plan = rte.Plan(spec, torch.float64)
    J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, Gm)
    torch.cuda.synchronize()
    f = floor_gradient(spec, Gm)
    errs = dict(G=rel(G.cpu(), G_o), J=abs(J.item() - J_o) / abs(J_o), ga=rel(ga.cpu(), ga_o), gb=rel(gb.cpu(), gb_o))
    say("  errors", {k: "%.2e (floor %.2e)" % (v, f[k]) for k, v in errs.items()})
    for k, v in errs.items():
        assert v < tol(f[k]), (k, v, f[k])


def test_mss_combinations_match_oracle(rte):
    # 3 generalised sources with staggered beams (Sec. 3.1), solved together
    base = W.small_problem(N=24, M=16, K=50, seed=8, n_in=1.4, L=1.0)
    beams = []
    for k, (x, y) in enumerate([(0.5, 0.0), (1.0, 0.5), (0.5, 1.0), (0.0, 0.3), (0.7, 0.0)]):
        b = W.beam_at(x, y, 0, 1, 0, 1, sigma_t=2.0, t0=6.0, sigma_x=0.2, tau=1.5 * k)
        b.group = k % 3
        beams.append(b)
    spec = base.with_(beams=beams)
    say("mss", spec.Nq)
    o = Oracle(spec)
    Gm = _measured(o.forward()[0], 9)
    J_o, ga_o, gb_o, G_o = o.gradient(Gm)
    plan = rte.Plan(spec, torch.float64)
    J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, Gm)
    assert G.shape == (3, len(spec.detectors), spec.K)
    f = floor_gradient(spec, Gm)
    errs = dict(G=rel(G.cpu(), G_o), J=abs(J.item() - J_o) / abs(J_o), ga=rel(ga.cpu(), ga_o), gb=rel(gb.cpu(), gb_o))
    say("  errors", {k: "%.2e (floor %.2e)" % (v, f[k]) for k, v in errs.items()})
    for k, v in errs.items():
        assert v < tol(f[k]), (k, v, f[k])


def test_checkpointed_replay_is_bitwise_equal(rte):
    spec = W.small_problem(N=20, M=16, K=47, seed=10, n_in=1.4)
    say("checkpoint replay")
    Gm = np.random.default_rng(3).standard_normal((1, len(spec.detectors), spec.K)) * 1e-3
    outs = []
    for ck in (0, 1, 5, 16, 47, 100):
        plan = rte.Plan(spec, torch.float64, ckpt_every=ck)
        J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, Gm)
        outs.append((J.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy(), G.cpu().numpy()))
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("case", [CASES[1], CASES[5], CASES[7], CASES[9], CASES[2]], ids=["16", "64", "48", "80", "13"])
def test_fp32_matches_fp64_oracle(rte, case):
    # FP32 node passes use vector lanes (4 slots of one group per lane): 1 to
    # 4 row tiles of 16 slots at compile time and 5 at run time, square and
    # rectangular grids, Fresnel and index-matched boundaries
    spec = _spec(case)
    say("fp32", case)
    o = Oracle(spec)
    Gm = _measured(o.forward()[0], 200)
    J_o, ga_o, gb_o, G_o = o.gradient(Gm)
    plan = rte.Plan(spec, torch.float32)
    J, ga, gb, G = plan.gradient(spec.mu_a, spec.mu_s, Gm)
    errs = dict(G=rel(G.cpu(), G_o), ga=rel(ga.cpu(), ga_o), gb=rel(gb.cpu(), gb_o))
    say("  fp32 errors", errs)
    for k, v in errs.items():
        assert v < TOL32, (k, v)


def test_autograd_function_matches_library_adjoint(rte):
    spec = W.small_problem(N=16, M=8, K=30, seed=11)
    say("autograd")
    o = Oracle(spec)
    G_o, _, st = o.forward(keep_states=True)
    rng = np.random.default_rng(12)
    Gbar = rng.standard_normal(G_o.shape)
    ga_o, gb_o = o.adjoint(Gbar, st)
    plan = rte.Plan(spec, torch.float64)
    a = torch.tensor(spec.mu_a, device="cuda", requires_grad=True)
    b = torch.tensor(spec.mu_s, device="cuda", requires_grad=True)
    G = rte.RTEFunction.apply(a, b, plan)
    (G * torch.tensor(Gbar, device="cuda")).sum().backward()
    ob = Oracle(spec, dense_derivative=True)
    G_b, _, st_b = ob.forward(keep_states=True)
    ga_b, gb_b = ob.adjoint(Gbar, st_b)
    assert rel(G.detach().cpu(), G_o) < tol(rel(G_b, G_o))
    assert rel(a.grad.cpu(), ga_o) < tol(rel(ga_b, ga_o)) and rel(b.grad.cpu(), gb_o) < tol(rel(gb_b, gb_o))


def test_plain_forward_config0_full_size(rte):
    # the plain FP64 forward workload (65x65 nodes, 16 ordinates, 200 steps)
    spec = W.config(0)
    say("config 0 full", spec.name)
    o = Oracle(spec)
    G_o, uK_o, _ = o.forward()
    plan = rte.Plan(spec, torch.float64)
    G, uK = plan.forward(spec.mu_a, spec.mu_s, want_u_final=True)
    fG, fu = floor_forward(spec)
    say("  G %.2e (floor %.2e)  u %.2e" % (rel(G.cpu(), G_o), fG, rel(uK.cpu(), uK_o)))
    assert rel(G.cpu(), G_o) < tol(fG)
    assert rel(uK.cpu(), uK_o) < TOL64


def test_gradient_workload_full_size_spot_checks(rte):
    # 257x257 nodes, 32 ordinates, 2000 steps in the same launch configuration
    # as the benchmark.  The oracle recomputes the first 12 steps in full; the
    # whole 2000-step gradient is checked by a directional derivative.
    spec = W.config(1)
    say("config 1 full", spec.name)
    plan = rte.Plan(spec, torch.float64)
    a = torch.tensor(spec.mu_a, device="cuda")
    b = torch.tensor(spec.mu_s, device="cuda")
    G0 = plan.forward(a, b).cpu().numpy()
    Gm = G0 * (1 + 0.1 * np.random.default_rng(2).standard_normal(G0.shape))
    J, ga, gb, G = plan.gradient(a, b, Gm)
    assert np.array_equal(G.cpu().numpy(), G0)
    # oracle on the first steps
    Ks = 12
    o = Oracle(spec.with_(K=Ks))
    G_o, uK_o, _ = o.forward()
    plan_s = rte.Plan(spec.with_(K=Ks), torch.float64)
    Gs, uKs = plan_s.forward(a, b, want_u_final=True)
    say("  first %d steps: u %.2e  G %.2e (|G| max %.1e)" % (Ks, rel(uKs.cpu(), uK_o), rel(Gs.cpu(), G_o) if np.abs(G_o).max() > 0 else 0.0, np.abs(G_o).max()))
    assert rel(uKs.cpu(), uK_o) < TOL64
    # (G of this run is compared element by element over 300 lit steps in
    # tests/test_gpu_fullsize.py; here the detectors are still dark)
    # directional derivative of J along a smooth perturbation
    rng = np.random.default_rng(5)
    X, Y = np.meshgrid(np.linspace(0, 1, spec.Nx + 1), np.linspace(0, 1, spec.Ny + 1))
    da = torch.tensor(np.sin(2 * math.pi * X) * np.cos(math.pi * Y) * spec.mu_a, device="cuda")
    db = torch.tensor(rng.uniform(-1, 1) * np.cos(3 * X) * spec.mu_s, device="cuda")
    ad = float((ga * da).sum() + (gb * db).sum())
    def Jat(eps):
        Ge = plan.forward(a + eps * da, b + eps * db).cpu().numpy()
        return 0.5 * spec.dt * np.sum((Ge - Gm) ** 2)
    eps = 1e-4
    fd = (Jat(eps) - Jat(-eps)) / (2 * eps)
    assert abs(fd - ad) < 1e-6 * abs(ad), (fd, ad)


def test_neck_phantom_first_steps(rte):
    # the neck phantom's own grid (1025 x 1025 nodes, 64 ordinates: x and y
    # lines of N_p = 1080 on the generic line kernel), one combination, the
    # first 3 steps, FP64 and FP32 against the FP64 oracle
    import dataclasses
    full = W.neck_phantom()
    spec = full.with_(K=3, beams=[dataclasses.replace(b, group=0, tau=0.0, t0=0.0) for b in full.beams if b.group == 0])
    say("neck first steps", spec.Nx + 1, spec.M, spec.K)
    _first_steps_check(rte, spec, Np=1080)


def test_mss_workload_first_steps(rte):
    # the batched MSS workload's own grid (513 x 513 nodes, 64 ordinates,
    # N_p = 540 four-step lines), two of its combinations solved together,
    # the first 3 steps, FP64 and FP32 against the FP64 oracle
    import dataclasses
    full = W.config(2)
    keep = {0: 0, 5: 1}
    spec = full.with_(K=3, beams=[dataclasses.replace(b, group=keep[b.group], tau=0.0, t0=0.0)
                                  for b in full.beams if b.group in keep])
    say("mss first steps", spec.Nx + 1, spec.M, spec.Nq, spec.K)
    _first_steps_check(rte, spec, Np=540, Nq=2)


@pytest.mark.parametrize("idx", [4, 9])
def test_uneven_instances_first_steps(rte, idx):
    # full-size instances of the uneven batch with 48 ordinates (3 row tiles
    # of 16 slots) on their own grids (330 and 481 nodes per side: N_p = 360
    # and 512), the first 3 steps, FP64 and FP32 against the FP64 oracle
    import dataclasses
    full = W.uneven_batch()[idx]
    spec = full.with_(K=3, beams=[dataclasses.replace(b, tau=0.0, t0=0.0) for b in full.beams])
    say("uneven instance", idx, spec.Nx + 1, spec.M)
    _first_steps_check(rte, spec)


def _first_steps_check(rte, spec, Np=None, Nq=None):
    """u^K by relative L2 to 1e-10 (1e-5 FP32); G by relative L2 against
    the oracle's G, within max(1e-10, 4 x floor) in FP64 (the pulses are
    moved to the start so that the detectors are lit)."""
    G_o, uK_o, _ = Oracle(spec).forward()
    fG, _ = floor_forward(spec)
    assert np.linalg.norm(G_o) > 0
    for dt, bar in ((torch.float64, TOL64), (torch.float32, TOL32)):
        plan = rte.Plan(spec, dt)
        if Np is not None:
            assert plan.Np_x == Np and plan.Np_y == Np
        if Nq is not None:
            assert plan.Nq == Nq
        G, uK = plan.forward(spec.mu_a, spec.mu_s, want_u_final=True)
        torch.cuda.synchronize()
        eu, eg = rel(uK.cpu(), uK_o), rel(G.cpu(), G_o)
        gbar = tol(fG) if dt == torch.float64 else bar
        say("  %s: N_p %d, u %.2e  G %.2e (floor %.2e)" % (dt, plan.Np_x, eu, eg, fG))
        assert eu < bar and eg < gbar, (eu, eg, gbar)
        plan.close()
