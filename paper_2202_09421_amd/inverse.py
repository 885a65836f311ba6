"""Outer inverse loop (Sec. 6, Algorithm algfcinv): box-constrained L-BFGS-B
over the nodal absorption a, objective eq. (FObjpr), gradient from the
library (one forward and one adjoint per generalised source per
evaluation), reconstruction error E(i) of eq. (errl2).

The optimiser is SciPy's L-BFGS-B (the limited-memory bound-constrained
quasi-Newton method of Byrd et al. that the paper cites).  The objective is
scaled by its value at the initial guess (a positive constant does not move
the minimiser; it keeps the projected gradient in the range L-BFGS-B's
stopping tests expect).  The scattering b stays fixed, as in the paper's
reconstructions.
"""
from __future__ import annotations

import time

import numpy as np


def relative_l2_error(a_true, a, dx, dy):
    """E = sqrt(int (a_t - a)^2 / int a_t^2), trapezoid rule on the nodes (eq. errl2)."""
    ny, nx = a_true.shape
    wy = np.full(ny, dy)
    wy[0] = wy[-1] = dy / 2
    wx = np.full(nx, dx)
    wx[0] = wx[-1] = dx / 2
    w = np.outer(wy, wx)
    return float(np.sqrt(np.sum(w * (a_true - a) ** 2) / np.sum(w * a_true ** 2)))


def plan_objective(plan, mu_s, G_meas, continuous=False, graph=False):
    """grad_fn(a) -> (J, dJ/da) on the host (float, [ny, nx] FP64) from
    Plan.gradient (exact discrete adjoint) or Plan.gradient_continuous.
    The medium lives in fixed device buffers, so with graph=True (exact
    adjoint only) every evaluation replays one recorded HIP graph."""
    import torch

    dev = plan.device
    ny, nx = plan.spec.Ny + 1, plan.spec.Nx + 1
    a_dev = torch.empty((ny, nx), dtype=plan.dtype, device=dev)
    b = torch.as_tensor(mu_s, dtype=plan.dtype, device=dev).contiguous()
    gm = torch.as_tensor(G_meas, dtype=torch.float64, device=dev).contiguous()
    if graph and not continuous:
        plan.set_graph(True)
    run = plan.gradient_continuous if continuous else plan.gradient

    def grad_fn(a):
        a_dev.copy_(torch.as_tensor(np.asarray(a, dtype=np.float64).reshape(ny, nx), dtype=plan.dtype))
        J, ga, _, _ = run(a_dev, b, gm)
        return float(J.item()), ga.detach().cpu().numpy().astype(np.float64)

    return grad_fn


def reconstruct(grad_fn, a0, lower, upper, max_iter=20, a_true=None, dx=1.0, dy=1.0, maxcor=10):
    """Minimise J over lower <= a <= upper from a0 with L-BFGS-B.

    Returns (a_final, history): one record per iteration (and one for the
    initial guess) with the iteration index, J, E(i) when a_true is given,
    the number of objective evaluations so far and the elapsed seconds."""
    from scipy.optimize import minimize

    shape = np.shape(a0)
    J0, _ = grad_fn(np.asarray(a0, dtype=np.float64))
    scale = 1.0 / J0 if J0 > 0 else 1.0
    state = {"evals": 1, "last": None}
    t0 = time.perf_counter()

    def fun(x):
        J, g = grad_fn(x.reshape(shape))
        state["evals"] += 1
        state["last"] = J
        return J * scale, g.ravel() * scale

    history = [{"iter": 0, "J": J0, "E": None if a_true is None else relative_l2_error(a_true, a0, dx, dy),
                "evals": 1, "seconds": 0.0}]

    def callback(x):
        history.append({"iter": len(history), "J": state["last"],
                        "E": None if a_true is None else relative_l2_error(a_true, x.reshape(shape), dx, dy),
                        "evals": state["evals"], "seconds": time.perf_counter() - t0})

    lo = np.broadcast_to(np.asarray(lower, dtype=np.float64), shape).ravel()
    hi = np.broadcast_to(np.asarray(upper, dtype=np.float64), shape).ravel()
    res = minimize(fun, np.asarray(a0, dtype=np.float64).ravel(), jac=True, method="L-BFGS-B",
                   bounds=list(zip(lo, hi)), callback=callback,
                   options={"maxiter": max_iter, "maxcor": maxcor, "ftol": 0.0, "gtol": 0.0})
    return res.x.reshape(shape), history
