"""Inputs of the manufactured-solution problem (Sec. 5, eqs. RTEdisp and
RTEmansol) for rte_forward_ex: u_an = exp(-(x - t)^2 - (y - t)^2 - cos^2 theta)
in a homogeneous isotropic medium (g = 0) with a plain inflow condition.

Substituting u_an in T[u] = (1/c) u_t + theta . grad u + (a + b) u
- b int eta u dtheta' gives a source of separable rank 3 in (x, t), (y, t),
theta with X1 = e^{-(x-t)^2}, X2 = (x - t) X1 (Y1, Y2 likewise) and
Th1 = e^{-cos^2 theta}:

    q = X2 Y1 [(2/c) Th1 - 2 cos(theta) Th1]
      + X1 Y2 [(2/c) Th1 - 2 sin(theta) Th1]
      + X1 Y1 [(a + b) Th1 - b k_Phi / (2 pi)],

k_Phi = int e^{-cos^2} = 2 pi e^{-1/2} I_0(1/2); the inflow data is u_an
itself (rank 1).  Host-side input construction only (numpy)."""
from __future__ import annotations

import math

import numpy as np


def k_phi():
    from scipy.special import i0
    return 2.0 * math.pi * math.exp(-0.5) * float(i0(0.5))


def manufactured_inputs(spec, a, b):
    """(u0, u_hist, source, inflow) for Plan.forward_ex, natural layouts, FP64."""
    nx, ny, M, K = spec.Nx + 1, spec.Ny + 1, spec.M, spec.K
    x = spec.xmin + spec.dx * np.arange(nx)
    y = spec.ymin + spec.dy * np.arange(ny)
    th = 2.0 * math.pi * np.arange(M) / M
    t = spec.dt * np.arange(-3, K + 1)                  # time levels -3..K
    ex = x[None, :] - t[:, None]
    ey = y[None, :] - t[:, None]
    X1, X2 = np.exp(-ex ** 2), ex * np.exp(-ex ** 2)
    Y1, Y2 = np.exp(-ey ** 2), ey * np.exp(-ey ** 2)
    T1 = np.exp(-np.cos(th) ** 2)
    c = spec.c
    source = (np.stack([X2, X1, X1]), np.stack([Y1, Y2, Y1]),
              np.stack([(2.0 / c) * T1 - 2.0 * np.cos(th) * T1,
                        (2.0 / c) * T1 - 2.0 * np.sin(th) * T1,
                        (a + b) * T1 - b * k_phi() / (2.0 * math.pi) * np.ones(M)]))
    inflow = (X1[None], Y1[None], T1[None])

    def state(level):
        k = level + 3
        return (Y1[k][:, None, None] * X1[k][None, :, None]) * T1[None, None, :]

    u0 = state(0)[None]
    u_hist = np.stack([state(-1)[None], state(-2)[None], state(-3)[None]])
    return u0, u_hist, source, inflow
