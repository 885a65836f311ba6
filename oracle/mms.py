"""Manufactured-solution problem (Sec. 5, eq. RTEdisp) on the oracle side
(test infrastructure only).

    T[u] = q in Omega x [0, 2 pi),  u(t = 0) = u0,  u = u_b on Gamma_-,
    u_an(x, theta, t) = exp(-(x - t)^2 - (y - t)^2 - cos(theta)^2)   (eq. RTEmansol)

with T[u] = (1/c) u_t + theta . grad u + (a + b) u - b int eta u dtheta'
(eq. RTE with homogeneous a, b).  q, u0 and u_b follow from substituting
u_an; the scattering integral of u_an is exact for an isotropic medium
(g = 0): int eta u_an = k_Phi / (2 pi) exp(-(x - t)^2 - (y - t)^2), with
k_Phi the printed constant (pinned against its closed form elsewhere).  The
paper's boundary here is a plain inflow condition (no Fresnel reflection:
n_in = n_out).  As in the paper, x - t mixes cm and ps; the source absorbs it.

Discretisation: the forward scheme of oracle.solver with q added to the
right-hand side (u_t = c (L(u) + q)), u^0 = u_an(0), the inflow entries set
to u_an(t_{n+1}) after every update, and the AB4 history started from the
exact solution: L^{-k} = L(u_an(t_{-k})) + q(t_{-k}), k = 1, 2, 3 (a reading:
the paper does not state its start-up; with it the start-up does not limit
the time order).  The error measure is the paper's: the maximum over the
nodes of |Phi_num(x, T) - Phi_an(x, T)|, Phi = int u dtheta (trapezoid rule
of eq. RTETrapz on the numerical side).
"""
from __future__ import annotations

import math

import numpy as np

from . import physics
from .solver import CHI

K_PHI = 4.052876133898710   # int_0^{2 pi} exp(-cos^2 theta) dtheta (Sec. 5)


def u_exact(o, t):
    X, Y = np.meshgrid(o.xs, o.ys)
    E = np.exp(-(X - t) ** 2 - (Y - t) ** 2)
    return E[..., None] * np.exp(-np.cos(o.theta) ** 2)[None, None, :]


def flux_exact(o, t):
    X, Y = np.meshgrid(o.xs, o.ys)
    return K_PHI * np.exp(-(X - t) ** 2 - (Y - t) ** 2)


def source(o, t, a, b):
    """q = T[u_an] for homogeneous a, b and an isotropic kernel."""
    X, Y = np.meshgrid(o.xs, o.ys)
    dx_, dy_ = (X - t)[..., None], (Y - t)[..., None]
    u = u_exact(o, t)
    c = o.spec.c
    u_t = 2.0 * (dx_ + dy_) * u
    grad_x, grad_y = -2.0 * dx_ * u, -2.0 * dy_ * u
    transport = np.cos(o.theta) * grad_x + np.sin(o.theta) * grad_y
    scat = (K_PHI / (2.0 * math.pi)) * np.exp(-(X - t) ** 2 - (Y - t) ** 2)[..., None]
    return u_t / c + transport + (a + b) * u - b * scat


def mms_forward(o, a, b, K=None):
    """u^K and the max flux error at T = K dt for homogeneous a, b (scalars)."""
    s = o.spec
    K = s.K if K is None else K
    if s.g != 0.0 or s.n_in != s.n_out:
        raise ValueError("the manufactured problem is isotropic with a plain inflow condition")
    A = np.full((o.ny, o.nx), float(a))
    B = np.full((o.ny, o.nx), float(b))
    cdt = s.c * s.dt
    hist = [o.L(u_exact(o, -k * s.dt), A, B) + source(o, -k * s.dt, a, b) for k in (1, 2, 3)]
    u = u_exact(o, 0.0)
    for n in range(K):
        t = n * s.dt
        Ln = o.L(u, A, B) + source(o, t, a, b)
        ut = u + cdt * (CHI[0] * Ln + CHI[1] * hist[0] + CHI[2] * hist[1] + CHI[3] * hist[2])
        ub = u_exact(o, (n + 1) * s.dt)
        u = ut.copy()
        u[o.bj, o.bi, o.bm] = ub[o.bj, o.bi, o.bm]
        hist = [Ln, hist[0], hist[1]]
    err = np.abs(physics.scalar_flux(u) - flux_exact(o, K * s.dt)).max()
    return u, err
