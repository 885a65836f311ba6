"""Continuous-adjoint gradient (oracle side; test infrastructure only).

The paper obtains the functional gradient from the adjoint back-transport
problem (eq. AdjointProblem) and the integral of lambda u (eq. gradient_fin),
discretised as eq. (FDwin22):

    T*[lambda] = -(1/c) d_t lambda - theta . grad lambda + (a + b) lambda
                 - b int eta lambda dtheta' = 0,       lambda(T) = 0,
    lambda = f lambda(theta_r) + sum_j (G_j - G~_j)(1 - f) w(|x - x_j| / sigma_d)
                                                        on Gamma_+,
    dg/da_l ~ -sum_{m, j} lambda_{l,m,j} u_{l,m,j} dtheta dx dy dt.

With s = T - t and reversed ordinates, psi(x, theta, s) = lambda(x, theta + pi,
T - s) satisfies the forward RTE (the HG kernel depends on theta . theta' only)
with zero initial data and an inflow condition on Gamma_- of the same form as
the forward one: Fresnel reflection through the same reflection map, plus the
detector residual as boundary source.  The oracle therefore solves psi with its
forward stepping (FC-DOM + AB4 + strong inflow condition), as the paper solves
the adjoint "by the same machinery".  Readings (the paper is silent on the
discrete details):

* psi^0 = 0 with zero AB4 history; the inflow source of psi^{k+1} (time
  s_{k+1}, i.e. t_{K-k-1}) is r(t_{K-k-1}) with r(t_n) = G^n - G~^n for
  n = 1..K and r(t_0) = 0;
* on an inflow entry (node b, ordinate m) the source is
  (1 - coef_a - coef_b) sum_j w(|x_b - x_j| / sigma_d) r_j: 1 - f of the wall
  the inflow rule selects (corner ties: both walls, equal f);
* time quadrature: lambda(t_j) = psi^{K-j} paired with u^j, rectangle rule
  over j (the terms j = 0 and j = K vanish: u^0 = 0, lambda(T) = 0);
* dg/db_l ~ -sum lambda (u - W u) dtheta dx dy dt, from
  dT/db[db] = db (u - int eta u) (the paper derives only a).

Against the exact derivative of the discrete misfit (oracle.solver adjoint)
this gradient agrees to discretisation error, not to rounding: its tests
check convergence under refinement.
"""
from __future__ import annotations

import math

import numpy as np

from . import physics
from .solver import CHI


def residual_source_table(o, r):
    """Inflow source of psi on the oracle's BC entries for every time level.

    r: [Nd, K] residual G - G~ of one source (r[:, n-1] at t_n).  Returns
    S [K+1, n_bc] with S[k] the source at s_k = t_{K-k} (S[K] = r(t_0) = 0)."""
    s = o.spec
    xb = o.xs[o.bi]
    yb = o.ys[o.bj]
    wd = np.zeros((len(s.detectors), len(o.bm)))
    for jd, det in enumerate(s.detectors):
        wd[jd] = physics.window(np.hypot(xb - det.x, yb - det.y) / det.sigma_d)
    one_minus_f = 1.0 - o.coef_a - o.coef_b
    K = r.shape[1]
    S = np.zeros((K + 1, len(o.bm)))
    for k in range(K):
        n = K - k                      # s_k = t_{K-k}
        S[k] = one_minus_f * (r[:, n - 1] @ wd)
    return S


def continuous_gradient(o, Gmeas, mu_a=None, mu_s=None, G_res=None):
    """J, dg/da, dg/db (summed over sources) and G, by the continuous adjoint.
    G_res (tests only): traces to form the residual with instead of the
    oracle's own G (to drive the adjoint with another solver's traces)."""
    s = o.spec
    a = s.mu_a if mu_a is None else mu_a
    b = s.mu_s if mu_s is None else mu_s
    G, _, states = o.forward(a, b, keep_states=True)
    J = o.misfit(G, Gmeas)
    Gr = G if G_res is None else np.asarray(G_res, dtype=np.float64)
    K, M = s.K, s.M
    cdt = s.c * s.dt
    quad = (2.0 * math.pi / M) * s.dx * s.dy * s.dt
    ga = np.zeros((o.ny, o.nx))
    gb = np.zeros((o.ny, o.nx))
    for q in range(s.Nq):
        S = residual_source_table(o, Gr[q] - Gmeas[q])
        psi = np.zeros((o.ny, o.nx, M))
        hist = [np.zeros_like(psi) for _ in range(3)]
        for k in range(K):
            # lambda(t_{K-k}) = psi^k (reversed ordinates) with u^{K-k}
            u_rev = np.roll(states[q][K - k], -(M // 2), axis=-1)   # u at theta + pi
            Wpsi = psi @ o.W.T
            ga -= quad * np.sum(psi * u_rev, axis=-1)
            gb += quad * np.sum((Wpsi - psi) * u_rev, axis=-1)
            Lk = o.L(psi, a, b)
            pt = psi + cdt * (CHI[0] * Lk + CHI[1] * hist[0] + CHI[2] * hist[1] + CHI[3] * hist[2])
            psi = pt.copy()
            psi[o.bj, o.bi, o.bm] = (o.coef_a * pt[o.bj, o.bi, o.src_a] + o.coef_b * pt[o.bj, o.bi, o.src_b]
                                     + S[k + 1])
            hist = [Lk, hist[0], hist[1]]
    return J, ga, gb, G
