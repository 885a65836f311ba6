"""Pins of the oracle's time stepping, boundary treatment and adjoint against
exact solutions, invariants and brute force (Sec. 2, 3.4-3.6, 4.1-4.2)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import physics
from oracle.solver import CHI, Oracle
from tests.golden.values import paper_values

PV = paper_values()


def test_ab4_weights_consistent_with_printed_values():
    # Sec. 4.2 prints chi_1, chi_2 and chi_3 (as "chi_4"); chi_0 is garbled
    assert CHI[1] == PV["ab4_chi1"] and CHI[2] == PV["ab4_chi2"] and CHI[3] == PV["ab4_chi3"]
    assert abs(CHI.sum() - 1.0) < 1e-15  # consistency fixes chi_0 = 55/24
    # fourth order: the weights integrate 1, s, s^2, s^3 exactly over [0, 1]
    # with nodes at s = 0, -1, -2, -3
    s = -np.arange(4.0)
    for p in range(4):
        assert abs(np.sum(CHI * s ** p) - 1.0 / (p + 1)) < 1e-14


def _free_streaming(N, M=8):
    L, s0 = 1.0, 0.12
    x0 = np.array([-0.75, 0.5])
    spec = W.small_problem(N=N, M=M, K=1, L=L, a0=0.0, b0=0.0, n_in=1.0, heterogeneous=False)
    spec = spec.with_(mu_a=np.zeros_like(spec.mu_a), mu_s=np.zeros_like(spec.mu_s), n_in=1.0, n_out=1.0)
    T = 1.0 / spec.c
    K = int(round(T / spec.dt))
    spec = spec.with_(K=K, dt=T / K)
    o = Oracle(spec)
    th = o.theta

    def exact(X, Y, thm, t):
        px = X - spec.c * np.cos(thm) * t - x0[0]
        py = Y - spec.c * np.sin(thm) * t - x0[1]
        return np.exp(-(px ** 2 + py ** 2) / (2 * s0 ** 2))

    o.inflow = lambda t: exact(o.xs[o.bi], o.ys[o.bj], th[o.bm], t)
    _, uK, _ = o.forward()
    X, Y = np.meshgrid(o.xs, o.ys)
    ex = exact(X[..., None], Y[..., None], th[None, None, :], T)
    return np.max(np.abs(uK[0] - ex))


def test_free_streaming_matches_exact_advection():
    # a = b = 0, no reflection, inflow data = exact solution of the transport
    # equation: the discrete solution converges to exact advection at high order
    e1, e2 = _free_streaming(24), _free_streaming(48)
    assert e2 < 2e-3 and e1 / e2 > 8.0, (e1, e2)


@pytest.mark.parametrize("k", [0, 1, 3])
def test_uniform_state_decays_like_scalar_ab4(k):
    # spatially uniform state with angular mode k: the scheme reduces to the
    # scalar AB4 recurrence with rate c (a + b (1 - p_k)), p_k the closed-form
    # eigenvalue of the exponent-1 HG matrix
    M, g, a, b = 16, 0.6, 0.4, 8.0
    spec = W.small_problem(N=12, M=M, K=120, a0=a, b0=b, g=g, n_in=1.0, heterogeneous=False, hg_exponent=1.0)
    spec = spec.with_(n_out=1.0)
    o = Oracle(spec)
    pk = (g ** k + g ** (M - k)) / (1 + g ** M)
    lam = spec.c * (a + b * (1 - pk))
    prof = np.cos(k * o.theta)
    y = [1.0]
    f = [0.0, 0.0, 0.0]  # zero history
    for n in range(spec.K):
        fn = -lam * y[-1]
        y.append(y[-1] + spec.dt * (CHI[0] * fn + CHI[1] * f[0] + CHI[2] * f[1] + CHI[3] * f[2]))
        f = [fn, f[0], f[1]]
    y = np.array(y)
    o.inflow = lambda t: y[int(round(t / spec.dt))] * prof[o.bm]
    u0 = np.ones((13, 13, 1)) * prof[None, None, :]
    _, uK, _ = o.forward(u0=u0)
    assert np.max(np.abs(uK[0] - y[-1] * prof)) < 1e-8
    # and the recurrence follows exp(-lam t)
    # (zero history makes the start-up first order: a ~1% offset, while a
    # wrong weight, sign or rate would change the decay completely)
    assert abs(y[-1] - math.exp(-lam * spec.K * spec.dt)) < 2e-2 * math.exp(-lam * spec.K * spec.dt)


def _rot(u, N, M):
    """90-degree counter-clockwise rotation of a field u[j, i, m] on a square grid."""
    j, i, m = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(M), indexing="ij")
    out = np.empty_like(u)
    out[i, N - j, (m + M // 4) % M] = u[j, i, m]
    return out


def _rot2(a, N):
    j, i = np.meshgrid(np.arange(N + 1), np.arange(N + 1), indexing="ij")
    out = np.empty_like(a)
    out[i, N - j] = a[j, i]
    return out


@pytest.mark.parametrize("M", [8, 16])
def test_rotation_equivariance(M):
    # D4 symmetry of the square: rotating medium and field rotates L(u) and the
    # boundary map (pins signs of xi/eta, D_x/D_y and the corner rule)
    N = 14
    spec = W.small_problem(N=N, M=M, K=1, seed=5, n_in=1.4)
    o = Oracle(spec)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((N + 1, N + 1, M))
    a, b = spec.mu_a, spec.mu_s
    ra, rb = _rot2(a, N), _rot2(b, N)
    assert np.allclose(o.L(_rot(u, N, M), ra, rb), _rot(o.L(u, a, b), N, M), atol=1e-10 * np.abs(o.L(u, a, b)).max())
    o.inflow = lambda t: np.zeros(len(o.bm))
    assert np.allclose(o.apply_bc(_rot(u, N, M), 0, 0.0), _rot(o.apply_bc(u, 0, 0.0), N, M), atol=1e-15)


def test_scattering_conserves_ordinate_sum():
    spec = W.small_problem(N=10, M=16, K=1)
    o = Oracle(spec)
    u = np.random.default_rng(2).standard_normal((11, 11, 16))
    assert np.allclose((u @ o.W.T).sum(-1), u.sum(-1), atol=1e-13)


def test_mss_superposition():
    # MSS (Sec. 3.1): a combination of staggered beams gives the sum of the
    # single-beam detector traces (the RTE is linear in q)
    b1 = W.beam_at(0.5, 0.0, 0, 1, 0, 1, sigma_t=2.0, t0=6.0, sigma_x=0.2, tau=0.0)
    b2 = W.beam_at(1.0, 0.4, 0, 1, 0, 1, sigma_t=2.0, t0=6.0, sigma_x=0.2, tau=3.0)
    base = W.small_problem(N=12, M=8, K=80, seed=3)
    sep = base.with_(beams=[b1, W.Beam(**{**b2.__dict__, "group": 1})])
    comb = base.with_(beams=[b1, b2])
    Gs = Oracle(sep).forward()[0]
    Gc = Oracle(comb).forward()[0]
    assert np.allclose(Gc[0], Gs[0] + Gs[1], atol=1e-14 * np.abs(Gc).max())
    assert np.abs(Gs[1]).max() > 0.05 * np.abs(Gs[0]).max()


def test_long_run_stays_bounded():
    spec = W.small_problem(N=16, M=8, K=2500, seed=4, n_in=1.4)
    G, uK, _ = Oracle(spec).forward()
    assert np.all(np.isfinite(uK))
    peak = np.abs(G).max()
    assert peak > 0 and np.abs(G[..., -100:]).max() < 1e-2 * peak


def test_dot_product_identity():
    # <A u0, r> = <u0, A^T r> for the linear map from the initial state to the
    # detector traces (sources off): the adjoint is the exact transpose
    spec = W.small_problem(N=11, M=8, K=25, seed=6, n_in=1.4)
    o = Oracle(spec)
    o.inflow = lambda t: np.zeros(len(o.bm))
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal((12, 12, 8))
    G, _, states = o.forward(u0=u0, keep_states=True)
    r = rng.standard_normal(G.shape)
    _, _, u0bar = o.adjoint(r, states, want_u0bar=True)
    lhs = np.sum(G * r)
    rhs = np.sum(u0 * u0bar[0])
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + np.abs(G).max() * np.abs(r).sum())


def _measured(o, seed):
    G = o.forward()[0]
    rng = np.random.default_rng(seed)
    return G * (1 + 0.3 * rng.standard_normal(G.shape)) + 0.05 * np.abs(G).max() * rng.standard_normal(G.shape)


def test_gradient_matches_fd_on_every_node():
    spec = W.small_problem(N=10, M=8, K=24, seed=8, n_in=1.4, L=0.5)
    o = Oracle(spec)
    Gm = _measured(o, 9)
    J, ga, gb, _ = o.gradient(Gm)
    for grad, field in ((ga, "mu_a"), (gb, "mu_s")):
        base = getattr(spec, field)
        fd = np.zeros_like(base)
        for j in range(base.shape[0]):
            for i in range(base.shape[1]):
                def central(eps):
                    p, m = base.copy(), base.copy()
                    p[j, i] += eps
                    m[j, i] -= eps
                    args_p = (p, None) if field == "mu_a" else (None, p)
                    args_m = (m, None) if field == "mu_a" else (None, m)
                    return (o.misfit(o.forward(*args_p)[0], Gm) - o.misfit(o.forward(*args_m)[0], Gm)) / (2 * eps)
                # Richardson-extrapolated centred differences (O(eps^4)); a step
                # of 1% keeps round-off in J far below the truncation error
                eps = 1e-2 * base[j, i]
                fd[j, i] = (4 * central(eps / 2) - central(eps)) / 3
        err = np.max(np.abs(fd - grad)) / np.max(np.abs(grad))
        assert err < 1e-7, (field, err)


def test_directional_fd_second_order():
    spec = W.small_problem(N=12, M=8, K=40, seed=10, n_in=1.4)
    o = Oracle(spec)
    Gm = _measured(o, 11)
    J, ga, gb, _ = o.gradient(Gm)
    rng = np.random.default_rng(12)
    da, db = rng.standard_normal(ga.shape) * spec.mu_a, rng.standard_normal(gb.shape) * spec.mu_s
    ad = np.sum(ga * da) + np.sum(gb * db)
    errs = []
    for eps in (1e-2, 1e-3):
        Jp = o.misfit(o.forward(spec.mu_a + eps * da, spec.mu_s + eps * db)[0], Gm)
        Jm = o.misfit(o.forward(spec.mu_a - eps * da, spec.mu_s - eps * db)[0], Gm)
        errs.append(abs((Jp - Jm) / (2 * eps) - ad) / abs(ad))
    assert errs[1] < 1e-6 and errs[0] / errs[1] > 50, errs
