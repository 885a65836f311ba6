"""The outer inverse loop (Sec. 6, Algorithm algfcinv) on the host, driven by
the oracle's gradient on a tiny phantom: the misfit never increases over the
accepted iterates, the box a^l <= a <= a^u holds, the reconstruction error
E(i) (eq. errl2) decreases, and E itself matches its closed form on a
constant field."""
import numpy as np

import workloads as W
from oracle.solver import Oracle
from paper_2202_09421_amd.inverse import reconstruct, relative_l2_error


def test_relative_l2_error_closed_form():
    a_t = np.full((5, 7), 2.0)
    assert relative_l2_error(a_t, a_t, 0.1, 0.2) == 0.0
    assert abs(relative_l2_error(a_t, 1.5 * a_t, 0.1, 0.2) - 0.5) < 1e-15
    # trapezoid weights: a perturbation on the boundary counts half
    a = a_t.copy()
    a[0, 3] += 1.0
    assert abs(relative_l2_error(a_t, a, 1.0, 1.0) ** 2 - 0.5 / (4.0 * 24.0)) < 1e-15


def test_lbfgsb_loop_with_oracle_gradient():
    spec = W.small_problem(N=12, M=8, K=60, seed=31, n_in=1.4, g=0.8, a0=0.2, b0=5.0)
    X, Y = np.meshgrid(np.linspace(0, 1, 13), np.linspace(0, 1, 13))
    a_true = 0.2 + 0.4 * np.exp(-((X - 0.5) ** 2 + (Y - 0.4) ** 2) / 0.02)
    spec = spec.with_(mu_a=a_true, mu_s=np.full_like(a_true, 5.0))
    o = Oracle(spec)
    Gm = o.forward()[0]

    def grad_fn(a):
        J, ga, _, _ = o.gradient(Gm, mu_a=a)
        return J, ga

    a0 = np.full_like(a_true, 0.2)
    a, hist = reconstruct(grad_fn, a0, 0.2, 1.0, max_iter=6, a_true=a_true, dx=spec.dx, dy=spec.dy)
    Js = [h["J"] for h in hist]
    assert all(J1 <= J0 * (1 + 1e-12) for J0, J1 in zip(Js, Js[1:])), Js
    assert Js[-1] < 0.5 * Js[0]
    assert a.min() >= 0.2 - 1e-15 and a.max() <= 1.0 + 1e-15
    assert hist[-1]["E"] < hist[0]["E"]
