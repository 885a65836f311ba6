"""Pins of the oracle's detector readout, eq. (OpMed), discretised with the
trapezoid rule along each wall and the DOM sum over outgoing ordinates.

For a uniform isotropic state u = 1 the reading factorises into an angular
factor and a spatial footprint integral:
  * angular: sum over strictly outgoing ordinates of (2 pi / M)(1 - f) theta.nu;
    with f = 0 this is (2 pi / M) cot(pi / M) exactly (a Dirichlet-kernel sum),
    and as M grows it tends to the integral of (1 - f(cos)) cos over the
    outgoing half circle, checked against an independent quadrature with the
    Fresnel law written in its angle form (Stokes' relations);
  * spatial: sum over walls of the trapezoid rule of w(|x_b - x_j| / sigma_d),
    which tends to the boundary integral of the footprint; for a detector
    whose footprint lies inside one wall, or sits exactly on a corner, the
    integrand extends evenly across the wall ends and the trapezoid rule with
    half weights at the ends is exact to round-off; a corner counted on both
    of its walls with half weight gives the full integral.
A dropped or doubled end weight, a corner read on one wall only, incoming
instead of outgoing ordinates, a missing cosine or 2 pi / M factor, or a
wrong spacing all move these numbers far outside the tolerances."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import workloads as W
from oracle import physics
from oracle.solver import Oracle


def _spec(Nx, Ny, M, dets, n_in=1.0, Lx=2.0, Ly=1.5):
    a = np.full((Ny + 1, Nx + 1), 0.1)
    return W.ProblemSpec(0.0, Lx, 0.0, Ly, Nx, Ny, M, 1, 0.01, a, a.copy(),
                         [W.Beam(Lx / 2, 0.0, math.pi / 2)], dets, n_in=n_in, n_out=1.0)


def _footprint_integral(det, Lx, Ly):
    """Boundary integral of w(|x - x_j| / sigma_d) over the four walls."""
    s = det.sigma_d
    f = lambda d: float(physics.window(np.array([d / s]))[0])
    walls = [(lambda t: (t, 0.0), Lx), (lambda t: (t, Ly), Lx), (lambda t: (0.0, t), Ly), (lambda t: (Lx, t), Ly)]
    tot = 0.0
    for pt, L in walls:
        g = lambda t: f(math.hypot(pt(t)[0] - det.x, pt(t)[1] - det.y))
        tot += quad(g, 0.0, L, limit=400, epsabs=1e-15, epsrel=1e-13,
                    points=[min(max(det.x if L == Lx else det.y, 0.0), L)])[0]
    return tot


def _uniform_reading(spec):
    o = Oracle(spec)
    return o.detect(np.ones((spec.Ny + 1, spec.Nx + 1, spec.M)))


def test_uniform_state_reading_equals_angular_factor_times_footprint_integral():
    Lx, Ly, M = 2.0, 1.5, 16
    dets = [W.Detector(1.0, 0.0), W.Detector(2.0, 0.75), W.Detector(0.0, 0.0), W.Detector(2.0, 1.5),
            W.Detector(0.7, 1.5)]
    # the trapezoid rule converges faster than any power for this smooth,
    # flat-ended footprint (3e-6, 8.5e-9, 8.5e-12 relative at 100, 200, 400
    # intervals per 2 cm); at 800 it is at round-off
    spec = _spec(800, 600, M, dets, Lx=Lx, Ly=Ly)
    G = _uniform_reading(spec)
    ang = (2 * math.pi / M) / math.tan(math.pi / M)
    for j, det in enumerate(dets):
        want = ang * _footprint_integral(det, Lx, Ly)
        assert abs(G[j] - want) <= 1e-13 * want, (j, G[j], want)
    # a mid-wall footprint integrates to 2 sigma_d int_0^1 w (one wall), and so
    # does a corner one (half of it on each wall)
    half = quad(lambda v: float(physics.window(np.array([v]))[0]), 0, 1, epsabs=1e-15)[0]
    for j in (0, 2, 3):
        assert abs(G[j] - ang * 2 * 0.3 * half) <= 1e-13 * G[j]


def test_near_corner_footprint_converges_at_second_order():
    # a footprint cut by a wall end is integrated with the trapezoid rule's
    # second-order end error; halving h divides the error by 4
    det = W.Detector(0.0, 0.1)
    want = (2 * math.pi / 8) / math.tan(math.pi / 8) * _footprint_integral(det, 2.0, 1.5)
    errs = []
    for N in (80, 160, 320):
        G = _uniform_reading(_spec(N, (3 * N) // 4, 8, [det]))
        errs.append(abs(G[0] - want) / want)
    assert errs[0] > 1e-7
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 < e0 / e1 < 4.4, errs


def _fresnel_stokes(theta_i, n1, n2):
    """Unpolarised reflectance from the angle form of the Fresnel amplitudes:
    r_s = -sin(ti - tt) / sin(ti + tt), r_p = tan(ti - tt) / tan(ti + tt)."""
    st = n1 / n2 * math.sin(theta_i)
    if st >= 1.0:
        return 1.0
    tt = math.asin(st)
    if theta_i == 0.0:
        return ((n1 - n2) / (n1 + n2)) ** 2
    rs = -math.sin(theta_i - tt) / math.sin(theta_i + tt)
    rp = math.tan(theta_i - tt) / math.tan(theta_i + tt)
    return 0.5 * (rs * rs + rp * rp)


def test_angular_factor_with_fresnel_converges_to_the_half_circle_integral():
    n = 1.4
    crit = math.asin(1.0 / n)
    # t = crit - s^2 removes the square-root edge of 1 - f at the critical angle
    exact = 2 * quad(lambda s: (1 - _fresnel_stokes(crit - s * s, n, 1.0)) * math.cos(crit - s * s) * 2 * s,
                     0, math.sqrt(crit), epsabs=1e-14, epsrel=1e-13, limit=200)[0]
    errs = []
    for M in (256, 1024, 4096):
        spec = _spec(12, 12, M, [W.Detector(1.0, 0.0)], n_in=n)
        xs = spec.xmin + spec.dx * np.arange(spec.Nx + 1)
        ys = spec.ymin + spec.dy * np.arange(spec.Ny + 1)
        for (w, wts, kappa) in physics.detector_tables(spec, xs, ys):
            errs.append((w.idx, M, abs(kappa.sum() - exact) / exact))
    for idx in range(4):
        e = [x[2] for x in errs if x[0] == idx]
        # 2e-3, 4.6e-5, 1.5e-6 at M = 256, 1024, 4096 (the square-root edge of
        # 1 - f at the critical angle limits the order)
        assert e[-1] < 1e-5, e
        assert e[0] / e[-1] > 100, e


def test_window_time_profile_closed_form():
    # eq. (sourcelab): T = w(|t - t_s| / sigma_t) with w(1/2) = exp(-4 e^-2),
    # w(0) = 1 and w = 0 from |t - t_s| = sigma_t on
    b = W.Beam(0.0, 0.0, 0.0, tau=5.0, t0=10.0, sigma_t=30.0, profile="window")
    t = np.array([15.0, 0.0, 30.0, 45.0, 45.0 + 1e-9, 100.0, -20.0])
    T = physics.beam_time(b, t)
    assert T[0] == 1.0
    assert abs(T[1] - math.exp(-4 * math.exp(-2))) < 1e-15
    assert abs(T[2] - math.exp(-4 * math.exp(-2))) < 1e-15
    assert T[3] == 0.0 and T[4] == 0.0 and T[5] == 0.0 and T[6] == 0.0
    g = W.Beam(0.0, 0.0, 0.0, tau=5.0, t0=10.0, sigma_t=30.0)
    assert abs(physics.beam_time(g, 45.0) - math.exp(-0.5)) < 1e-15
