"""Seeded synthetic workloads for the FC-DOM time-domain RTE solver.

This module only *describes* problems: grids, media, beams, detectors and
step counts, drawn from ``numpy.random.default_rng(seed)``.  It holds none of
the solver's arithmetic (no phase function, no Fresnel law, no continuation,
no time stepping), so both the FP64 CPU oracle and the HIP library consume
the same inputs without sharing any of the method's code.

Geometry follows the paper's setting (Sec. 2 and Sec. 4.3): a rectangle
[xmin,xmax] x [ymin,ymax], a uniform grid with Nx, Ny intervals (Nx+1, Ny+1
nodes), M ordinates theta_m = 2*pi*m/M, absorption a(x) = mu_a and scattering
b(x) = mu_s given on the nodes.  Units: cm, ps, 1/cm.

Beams follow eq. (RTEsources2) and the laboratory model eq. (sourcelab):
position on the boundary, direction (inward normal of its side), spatial
width sigma_x, angular width sigma_theta, temporal Gaussian of width sigma_t
centred at tau + t0.  Detectors follow eq. (OpMed): a boundary point and a
footprint sigma_d.  The multiple-staggered-source (MSS) combinations of
Sec. 3.1 are expressed with ``Beam.group``: beams of one group are fired in
the same generalised source q_i.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C_LIGHT = 0.0214  # cm/ps, average speed of light in tissue-like media (n ~ 1.4)


@dataclasses.dataclass
class Beam:
    x: float
    y: float
    theta: float          # beam direction (inward normal of its side)
    sigma_x: float = 0.3  # cm
    sigma_theta: float = math.pi / 4
    tau: float = 0.0      # ps, staggering delay
    sigma_t: float = 20.0  # ps
    t0: float = 60.0      # ps, pulse centre offset (3 sigma_t) so q(t<=0) ~ 0
    group: int = 0        # generalised source index i of q_i
    profile: str = "gauss"  # temporal profile: "gauss" or "window" (eq. sourcelab)


@dataclasses.dataclass
class Detector:
    x: float
    y: float
    sigma_d: float = 0.3  # cm


@dataclasses.dataclass
class ProblemSpec:
    """One instance of the discrete forward/adjoint problem (plain data)."""
    xmin: float
    xmax: float
    ymin: float
    ymax: float
    Nx: int               # intervals; Nx+1 nodes
    Ny: int
    M: int                # ordinates
    K: int                # time steps
    dt: float             # ps
    mu_a: np.ndarray      # [Ny+1, Nx+1] absorption a(x), 1/cm
    mu_s: np.ndarray      # [Ny+1, Nx+1] scattering b(x), 1/cm
    beams: List[Beam]
    detectors: List[Detector]
    c: float = C_LIGHT
    g: float = 0.9
    hg_exponent: float = 1.5
    n_in: float = 1.4
    n_out: float = 1.0
    fc_d: int = 5
    fc_C: int = 25
    filt_alpha: float = 2.0
    filt_beta: float = 55.0
    name: str = ""

    @property
    def Nq(self) -> int:
        return 1 + max((b.group for b in self.beams), default=0)

    @property
    def dx(self) -> float:
        return (self.xmax - self.xmin) / self.Nx

    @property
    def dy(self) -> float:
        return (self.ymax - self.ymin) / self.Ny

    @property
    def units(self) -> int:
        """cell * ordinate * step work units of one forward solve (all sources)."""
        return (self.Nx + 1) * (self.Ny + 1) * self.M * self.K * self.Nq

    def with_(self, **kw) -> "ProblemSpec":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------- helpers

def default_dt(dx: float, dy: float, c: float, mu_a: np.ndarray, mu_s: np.ndarray,
               cfl: float = 0.05, stiff: float = 0.1) -> float:
    """Time step recipe: dt = min(cfl*h/c, stiff/(c*max(a+b)))."""
    ext = float(np.max(mu_a + mu_s)) if np.size(mu_a) else 0.0
    dt = cfl * min(dx, dy) / c
    if ext > 0:
        dt = min(dt, stiff / (c * ext))
    return dt


def perimeter_point(s: float, xmin, xmax, ymin, ymax):
    """Point at arclength s counter-clockwise from (xmin, ymin) and the inward
    normal direction angle of its side."""
    Lx, Ly = xmax - xmin, ymax - ymin
    P = 2 * (Lx + Ly)
    s = s % P
    if s < Lx:
        return xmin + s, ymin, math.pi / 2
    s -= Lx
    if s < Ly:
        return xmax, ymin + s, math.pi
    s -= Ly
    if s < Lx:
        return xmax - s, ymax, 3 * math.pi / 2
    s -= Lx
    return xmin, ymax - s, 0.0


def perimeter_detectors(n_det: int, xmin, xmax, ymin, ymax, sigma_d=0.3) -> List[Detector]:
    P = 2 * ((xmax - xmin) + (ymax - ymin))
    out = []
    for j in range(n_det):
        x, y, _ = perimeter_point((j + 0.5) * P / n_det, xmin, xmax, ymin, ymax)
        out.append(Detector(x, y, sigma_d))
    return out


def beam_at(x, y, xmin, xmax, ymin, ymax, **kw) -> Beam:
    """Beam on the boundary point (x, y) pointing along the inward normal."""
    eps = 1e-12
    if abs(y - ymin) < eps:
        th = math.pi / 2
    elif abs(x - xmax) < eps:
        th = math.pi
    elif abs(y - ymax) < eps:
        th = 3 * math.pi / 2
    elif abs(x - xmin) < eps:
        th = 0.0
    else:
        raise ValueError("beam position must lie on the boundary")
    return Beam(x, y, th, **kw)


def _smooth_indicator(r: np.ndarray, radius: float, width: float) -> np.ndarray:
    """1 inside radius-width/2, 0 outside radius+width/2, quintic ramp between."""
    t = np.clip((radius + width / 2 - r) / width, 0.0, 1.0)
    return t * t * t * (10 - 15 * t + 6 * t * t)


def inclusions(rng, L: float, count: int, rmin=0.2, rmax=0.5, margin=0.5):
    """Non-overlapping discs with centres in [margin+r, L-margin-r]^2."""
    out = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > 10000:
            raise RuntimeError("could not place inclusions")
        r = rng.uniform(rmin, rmax)
        cx, cy = rng.uniform(margin + r, L - margin - r, size=2)
        if all(math.hypot(cx - x, cy - y) > r + rr for (x, y, rr) in out):
            out.append((cx, cy, r))
    return out


def grid_xy(xmin, xmax, ymin, ymax, Nx, Ny):
    x = xmin + (xmax - xmin) * np.arange(Nx + 1) / Nx
    y = ymin + (ymax - ymin) * np.arange(Ny + 1) / Ny
    return np.meshgrid(x, y)  # X[j,i], Y[j,i]


def inclusion_medium(L, N, a0, b0, seed, count=3, contrast=2.0):
    rng = np.random.default_rng(seed)
    X, Y = grid_xy(0.0, L, 0.0, L, N, N)
    h = L / N
    a = np.full(X.shape, a0)
    for (cx, cy, r) in inclusions(rng, L, count):
        ind = _smooth_indicator(np.hypot(X - cx, Y - cy), r, 2 * h)
        a = a + (contrast - 1.0) * a0 * ind
    b = np.full(X.shape, b0)
    return a, b


def measured_noise(rng_seed: int, shape, level=0.1) -> np.ndarray:
    """Multiplicative noise factors (1 + level*xi) for synthetic measurements."""
    rng = np.random.default_rng(rng_seed)
    return 1.0 + level * rng.standard_normal(shape)


# ---------------------------------------------------------------- configs

def config(idx: int) -> ProblemSpec:
    """The five benchmark configurations (0-based index)."""
    if idx == 0:
        L, N, M, K = 2.0, 64, 16, 200
        a = np.full((N + 1, N + 1), 0.1)
        b = np.full((N + 1, N + 1), 20.0)
        h = L / N
        return ProblemSpec(0, L, 0, L, N, N, M, K, default_dt(h, h, C_LIGHT, a, b), a, b,
                           [beam_at(1.0, 0.0, 0, L, 0, L)], perimeter_detectors(8, 0, L, 0, L),
                           g=0.8, n_in=1.0, n_out=1.0, name="plain-fp64-forward-64x64-M16")
    if idx == 1:
        L, N, M, K = 4.0, 256, 32, 2000
        a, b = inclusion_medium(L, N, 0.2, 50.0, seed=2)
        h = L / N
        return ProblemSpec(0, L, 0, L, N, N, M, K, default_dt(h, h, C_LIGHT, a, b), a, b,
                           [beam_at(2.0, 0.0, 0, L, 0, L)], perimeter_detectors(32, 0, L, 0, L),
                           g=0.9, n_in=1.4, name="fp64-gradient-256x256-M32-K2000")
    if idx == 2:
        L, N, M, K = 6.0, 512, 64, 6000
        a, b = inclusion_medium(L, N, 0.2, 50.0, seed=3)
        h = L / N
        rng = np.random.default_rng(3)
        taus = rng.uniform(0.0, 100.0, size=16)
        beams = []
        for j in range(16):
            x, y, th = perimeter_point((j + 0.5) * 1.5, 0, L, 0, L)
            beams.append(Beam(x, y, th, tau=float(taus[j]), group=j % 8))
        return ProblemSpec(0, L, 0, L, N, N, M, K, default_dt(h, h, C_LIGHT, a, b), a, b,
                           beams, perimeter_detectors(64, 0, L, 0, L), g=0.9, n_in=1.4,
                           name="mss-8x2-512x512-M64-K6000")
    if idx == 4:
        return neck_phantom()
    raise ValueError("config %d is a batch of instances; use uneven_batch()" % idx)


def uneven_batch(seed: int = 4, count: int = 32, scale: float = 1.0) -> List[ProblemSpec]:
    """Independent instances of uneven size (grids 128-512, M in {16,32,48,64},
    500-3000 steps, random smooth tissue maps).  ``scale`` shrinks grids and
    step counts for tests."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        N = int(rng.integers(128, 513))
        L = float(rng.uniform(2.0, 6.0))
        M = int(rng.choice([16, 32, 48, 64]))
        K = int(rng.integers(500, 3001))
        g = float(rng.uniform(0.7, 0.95))
        if scale != 1.0:
            N = max(16, int(N * scale))
            K = max(10, int(K * scale))
        X, Y = grid_xy(0, L, 0, L, N, N)
        a = np.full(X.shape, float(rng.uniform(0.05, 0.15)))
        b = np.full(X.shape, float(rng.uniform(20, 60)))
        for _ in range(4):
            cx, cy = rng.uniform(0.2 * L, 0.8 * L, size=2)
            s = rng.uniform(0.05 * L, 0.15 * L)
            bump = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
            a = a + rng.uniform(0.0, 0.3) * bump
            b = b + rng.uniform(0.0, 40.0) * bump
        a = np.clip(a, 0.05, 0.5)
        b = np.clip(b, 20.0, 100.0)
        h = L / N
        out.append(ProblemSpec(0, L, 0, L, N, N, M, K, default_dt(h, h, C_LIGHT, a, b), a, b,
                               [beam_at(L / 2, 0.0, 0, L, 0, L)], perimeter_detectors(16, 0, L, 0, L),
                               g=g, n_in=1.4, name="uneven-%d" % k))
    return out


def neck_phantom(N: int = 1024, K: int = 6000) -> ProblemSpec:
    """Layered neck-like phantom, 10 x 10 cm, 32 beams as 4 MSS combinations."""
    L = 10.0
    rng = np.random.default_rng(5)
    X, Y = grid_xy(0, L, 0, L, N, N)
    h = L / N
    a = np.full(X.shape, 0.1)
    b = np.full(X.shape, 40.0)
    # soft tissue with seeded variation
    a = a + 0.05 * np.sin(2 * math.pi * X / L * rng.uniform(0.5, 1.5)) * np.cos(2 * math.pi * Y / L * rng.uniform(0.5, 1.5))
    edge = np.minimum(np.minimum(X, L - X), np.minimum(Y, L - Y))
    band = _smooth_indicator(edge, 0.5, 2 * h)
    a = a * (1 - band) + 0.1 * band
    b = b * (1 - band) + 60.0 * band
    def ellipse(cx, cy, rx, ry):
        return _smooth_indicator(np.sqrt(((X - cx) / rx) ** 2 + ((Y - cy) / ry) ** 2), 1.0, 2 * h / min(rx, ry))
    bone = ellipse(5.0, 3.5, 1.2, 0.9)
    air = ellipse(5.0, 6.8, 0.8, 0.6)
    a = a * (1 - bone) + 0.4 * bone
    b = b * (1 - bone) + 120.0 * bone
    a = a * (1 - air) + 0.05 * air
    b = b * (1 - air) + 10.0 * air
    for (cx, cy, r) in inclusions(rng, L, 2, 0.3, 0.6, margin=1.5):
        t = _smooth_indicator(np.hypot(X - cx, Y - cy), r, 2 * h)
        a = a * (1 - t) + 0.3 * t
    a = np.clip(a, 0.05, 0.4)
    b = np.clip(b, 10.0, 120.0)
    taus = rng.uniform(0.0, 60.0, size=32)
    beams = []
    for j in range(32):
        x, y, th = perimeter_point((j + 0.5) * 1.25, 0, L, 0, L)
        beams.append(Beam(x, y, th, tau=float(taus[j]), group=j % 4))
    return ProblemSpec(0, L, 0, L, N, N, 64, K, default_dt(h, h, C_LIGHT, a, b), a, b, beams,
                       perimeter_detectors(128, 0, L, 0, L), g=0.9, n_in=1.4,
                       name="neck-1024x1024-M64-K6000")


def inverse_phantom(mode: str = "mss", N: int = 64, M: int = 16, seed: int = 6, n_beams: int = 8,
                    n_comb: int = 2, spacing: float = 40.0):
    """Inverse-problem test bed (Sec. 6 setting on a synthetic phantom):
    2 x 2 cm, background a = 0.1, b = 20 /cm, g = 0.8, Fresnel n = 1.4, two
    seeded inclusions with 3x absorption, n_beams beams evenly spaced on the
    perimeter, 16 detectors.  mode "ts": each beam is its own generalised
    source (T = 200 ps); "mss": n_comb combinations, beam j in combination
    j % n_comb, fired with delay spacing * (j // n_comb) (T = 200 ps plus
    the last delay).  Default: 8 beams, 2 combinations of 4 beams with
    delays 0, 40, 80, 120 ps (T = 320 ps).
    Returns (spec with the true medium, background a, lower bound a^l, upper
    bound a^u)."""
    L = 2.0
    rng = np.random.default_rng(seed)
    X, Y = grid_xy(0.0, L, 0.0, L, N, N)
    h = L / N
    a_bg, b_bg = 0.1, 20.0
    a = np.full(X.shape, a_bg)
    for (cx, cy, r) in inclusions(rng, L, 2, 0.2, 0.35, margin=0.4):
        a = a + 2.0 * a_bg * _smooth_indicator(np.hypot(X - cx, Y - cy), r, 2 * h)
    b = np.full(X.shape, b_bg)
    beams = []
    P = 4 * L
    for j in range(n_beams):
        x, y, th = perimeter_point((j + 0.5) * P / n_beams, 0, L, 0, L)
        if mode == "ts":
            beams.append(Beam(x, y, th, tau=0.0, group=j))
        else:
            beams.append(Beam(x, y, th, tau=spacing * (j // n_comb), group=j % n_comb))
    T = 200.0 if mode == "ts" else 200.0 + spacing * ((n_beams - 1) // n_comb)
    dt = default_dt(h, h, C_LIGHT, a, b)
    K = int(math.ceil(T / dt))
    spec = ProblemSpec(0, L, 0, L, N, N, M, K, dt, a, b, beams, perimeter_detectors(16, 0, L, 0, L),
                       g=0.8, n_in=1.4, name="inverse-%s-%dx%d-M%d" % (mode, N, N, M))
    return spec, np.full(X.shape, a_bg), a_bg, 1.0


def lab_flux(N: int = 200, M: int = 32, times=(30.0, 100.0, 170.0), dt: Optional[float] = None):
    """The laboratory photon-flux simulation of Sec. 5 (Fig. 6): [0,3]^2 cm,
    homogeneous a = 0.35 /cm, b = 20 /cm, g = 0.8, n = 1.4, one beam at
    (1.5, 0) along the inward normal (sigma_x = 0.3 cm, sigma_theta = pi/4)
    with the window time profile of eq. (sourcelab), t_s = 0 and
    sigma_t = 30 ps, as printed.  Returns (spec, steps):
    K reaches the last snapshot time and steps[k] is the time level nearest
    times[k]."""
    L = 3.0
    a = np.full((N + 1, N + 1), 0.35)
    b = np.full((N + 1, N + 1), 20.0)
    h = L / N
    if dt is None:
        dt = default_dt(h, h, C_LIGHT, a, b)
    steps = [int(round(t / dt)) for t in times]
    spec = ProblemSpec(0, L, 0, L, N, N, M, max(steps), dt, a, b,
                       [beam_at(1.5, 0.0, 0, L, 0, L, sigma_t=30.0, t0=0.0, profile="window")],
                       perimeter_detectors(4, 0, L, 0, L),
                       g=0.8, n_in=1.4, name="lab-flux-%dx%d-M%d" % (N, N, M))
    return spec, steps


def small_problem(N=16, M=8, K=40, L=1.0, g=0.5, n_in=1.4, a0=0.5, b0=5.0, seed=0,
                  n_det=4, beams=None, hg_exponent=1.5, heterogeneous=True, Ny=None,
                  dt=None) -> ProblemSpec:
    """Tiny seeded problem for unit tests (the oracle finishes in well under a second)."""
    rng = np.random.default_rng(seed)
    Ny = N if Ny is None else Ny
    Ly = L * Ny / N
    X, Y = grid_xy(0, L, 0, Ly, N, Ny)
    a = np.full(X.shape, a0)
    b = np.full(X.shape, b0)
    if heterogeneous:
        cx, cy = rng.uniform(0.3, 0.7, size=2)
        bump = np.exp(-((X / L - cx) ** 2 + (Y / Ly - cy) ** 2) / 0.02)
        a = a * (1 + rng.uniform(0.5, 1.5) * bump)
        b = b * (1 + rng.uniform(-0.3, 0.3) * bump)
    if beams is None:
        beams = [beam_at(0.5 * L, 0.0, 0, L, 0, Ly, sigma_t=2.0, t0=6.0, sigma_x=0.2 * L)]
    h = min(L / N, Ly / Ny)
    # the pulse must fit in the run: use a tiny time scale for tiny problems
    if dt is None:
        dt = default_dt(L / N, Ly / Ny, C_LIGHT, a, b)
    return ProblemSpec(0, L, 0, Ly, N, Ny, M, K, dt, a, b, beams,
                       perimeter_detectors(n_det, 0, L, 0, Ly, sigma_d=0.3 * L),
                       g=g, n_in=n_in, hg_exponent=hg_exponent, name="small")
