"""Ordinates, scattering, Fresnel boundary map, beams and detectors (oracle).

Passages followed:
  ordinates / quadrature       Sec. 4.1, eq. (RTETrapz): theta_m = 2 pi m / M,
                               weights 2 pi / M (0-based m here).
  Henyey-Greenstein            Sec. 2, eq. (Henyey-Greeinstein), with the
                               numerical normalisation of Sec. 4.1 (trapezoid
                               integral of the kernel equals one).
  boundary condition           Sec. 2, eq. (RTE), last line: on Gamma_- the
                               intensity equals f(theta.nu) u(theta_r) + q, with
                               theta_r = 2 theta_nu - theta + pi.
  window function              Sec. 2, eq. (sourcelabwind).
  beams                        Sec. 3.1, eqs. (RTEsources), (RTEsources2);
                               Sec. 5 eq. (sourcelab).
  detectors                    Sec. 3.1, eq. (OpMed).

Readings where the paper is silent:
  * Fresnel reflectance: the textbook unpolarised law from Snell's law with
    n_in inside and n_out outside, total reflection beyond the critical angle.
  * HG exponent: the printed 3/2 (kept as a parameter).
  * Corners: an ordinate incoming through both walls of a corner follows the
    wall with the larger |theta.nu|; on an exact tie the two walls' reflection
    terms are averaged.  Tangential ordinates (theta.nu = 0) get no condition.
  * Source time profile: exp(-(t - tau - t0)^2 / (2 sigma_t^2)), or, for a
    beam whose profile is "window", the window of eq. (sourcelabwind) in
    |t - t_s| / sigma_t with t_s = tau + t0 (eq. sourcelab).
  * Detector quadrature: trapezoid along each wall (half weight at the two end
    nodes of a wall), DOM sum over strictly outgoing ordinates.
Signs of theta.nu are decided with integer arithmetic on m so that the
ordinates parallel to a wall are classified exactly.
"""
from __future__ import annotations

import math

import numpy as np


# ------------------------------------------------------------------ ordinates

def ordinates(M: int):
    th = 2.0 * np.pi * np.arange(M) / M
    return th, np.cos(th), np.sin(th)


def scalar_flux(u: np.ndarray) -> np.ndarray:
    """eq. (photondensity) with the trapezoid rule of eq. (RTETrapz): the last
    axis holds the M ordinates."""
    M = u.shape[-1]
    return (2.0 * np.pi / M) * np.sum(u, axis=-1)


def cos_sign(m: int, M: int) -> int:
    """sign(cos(2 pi m / M)) exactly."""
    r = (4 * m) % (4 * M)
    if r == M or r == 3 * M:
        return 0
    return 1 if (r < M or r > 3 * M) else -1


def sin_sign(m: int, M: int) -> int:
    """sign(sin(2 pi m / M)) exactly."""
    r = (2 * m) % (2 * M)
    if r == 0 or r == M:
        return 0
    return 1 if r < M else -1


def x_dominates(m: int, M: int) -> int:
    """+1 if |cos theta_m| > |sin theta_m|, -1 if smaller, 0 on a tie."""
    mp_ = m % (M // 2)
    if 8 * mp_ == M or 8 * mp_ == 3 * M:
        return 0
    return 1 if (8 * mp_ < M or 8 * mp_ > 3 * M) else -1


# ------------------------------------------------------------------ scattering

def hg_matrix(M: int, g: float, exponent: float = 1.5) -> np.ndarray:
    """W[m, m'] = w_{m'} p_{m,m'}: HG kernel normalised so each row sums to one."""
    k = np.arange(M // 2 + 1)
    mu = np.cos(2.0 * np.pi * k / M)
    half = (1.0 - g * g) / (1.0 + g * g - 2.0 * g * mu) ** exponent
    p = np.concatenate([half, half[1:M - M // 2][::-1]])  # p[k] = p[M-k]
    p = p / p.sum()
    W = np.empty((M, M))
    for m in range(M):
        for mm in range(M):
            W[m, mm] = p[(m - mm) % M]
    return W


# ------------------------------------------------------------------ Fresnel

def fresnel(cos_i: float, n_in: float, n_out: float) -> float:
    """Unpolarised reflectance for a ray inside (index n_in) hitting the wall
    with |cos(angle to the normal)| = cos_i; transmission into n_out."""
    if n_in == n_out:
        return 0.0
    cos_i = min(max(cos_i, 0.0), 1.0)
    sin_i = math.sqrt(max(0.0, 1.0 - cos_i * cos_i))
    sin_t = n_in / n_out * sin_i
    if sin_t >= 1.0:
        return 1.0
    cos_t = math.sqrt(1.0 - sin_t * sin_t)
    rs = (n_in * cos_i - n_out * cos_t) / (n_in * cos_i + n_out * cos_t)
    rp = (n_out * cos_i - n_in * cos_t) / (n_out * cos_i + n_in * cos_t)
    return 0.5 * (rs * rs + rp * rp)


# ------------------------------------------------------------------ window

def window(v):
    """eq. (sourcelabwind)."""
    v = np.abs(np.asarray(v, dtype=np.float64))
    out = np.zeros_like(v)
    inside = (v > 0) & (v < 1)
    vi = v[inside]
    out[inside] = np.exp(2.0 * np.exp(-1.0 / vi) / (vi - 1.0))
    out[v == 0] = 1.0
    return out


def angular_distance(a, b):
    d = np.abs(np.mod(np.asarray(a) - b, 2.0 * np.pi))
    return np.minimum(d, 2.0 * np.pi - d)


# ------------------------------------------------------------------ walls

class Wall:
    """One side of the rectangle: its nodes (j, i), outward normal, spacing."""

    def __init__(self, idx, js, is_, nu, ds, x_wall):
        self.idx = idx
        self.js = np.asarray(js)
        self.is_ = np.asarray(is_)
        self.nu = nu
        self.ds = ds
        self.x_wall = x_wall  # True for x = const walls

    def dot_sign(self, m, M):
        """sign(theta_m . nu) exactly."""
        if self.x_wall:
            return cos_sign(m, M) * int(np.sign(self.nu[0]))
        return sin_sign(m, M) * int(np.sign(self.nu[1]))

    def dot(self, m, M):
        th = 2.0 * math.pi * m / M
        return math.cos(th) * self.nu[0] + math.sin(th) * self.nu[1]

    def reflect(self, m, M):
        """theta_r = 2 theta_nu - theta + pi as an ordinate index."""
        return (M // 2 - m) % M if self.x_wall else (-m) % M


def walls(Nx, Ny, dx, dy):
    jj = np.arange(Ny + 1)
    ii = np.arange(Nx + 1)
    return [
        Wall(0, jj, np.zeros_like(jj), (-1.0, 0.0), dy, True),    # x = xmin
        Wall(1, jj, np.full_like(jj, Nx), (1.0, 0.0), dy, True),  # x = xmax
        Wall(2, np.zeros_like(ii), ii, (0.0, -1.0), dx, False),   # y = ymin
        Wall(3, np.full_like(ii, Ny), ii, (0.0, 1.0), dx, False),  # y = ymax
    ]


def boundary_conditions(Nx, Ny, M, dx, dy, n_in, n_out):
    """All (node, ordinate) entries overwritten by the inflow condition.

    Returns arrays (j, i, m, src_a, coef_a, src_b, coef_b): the new value is
    coef_a * u~[j,i,src_a] + coef_b * u~[j,i,src_b] + q.  coef_b = 0 except on
    exact corner ties.
    """
    W4 = walls(Nx, Ny, dx, dy)
    per_node = {}
    for w in W4:
        for (j, i) in zip(w.js.tolist(), w.is_.tolist()):
            per_node.setdefault((j, i), []).append(w)
    rows = []
    for (j, i), ws in sorted(per_node.items()):
        for m in range(M):
            inc = [w for w in ws if w.dot_sign(m, M) < 0]
            if not inc:
                continue
            if len(inc) == 2:
                xs = [w for w in inc if w.x_wall][0]
                ys = [w for w in inc if not w.x_wall][0]
                dom = x_dominates(m, M)
                if dom > 0:
                    inc = [xs]
                elif dom < 0:
                    inc = [ys]
            terms = []
            for w in inc:
                f = fresnel(abs(w.dot(m, M)), n_in, n_out)
                terms.append((w.reflect(m, M), f / len(inc)))
            if len(terms) == 1:
                terms.append((m, 0.0))
            rows.append((j, i, m, terms[0][0], terms[0][1], terms[1][0], terms[1][1]))
    arr = np.array(rows, dtype=np.float64)
    return (arr[:, 0].astype(int), arr[:, 1].astype(int), arr[:, 2].astype(int),
            arr[:, 3].astype(int), arr[:, 4], arr[:, 5].astype(int), arr[:, 6])


# ------------------------------------------------------------------ beams

def beam_spatial_angular(beam, xb, yb, theta_m):
    """exp(-|x - x_k|^2 / (2 sigma_x^2)) * w(|theta - theta_k| / sigma_theta)."""
    r2 = (xb - beam.x) ** 2 + (yb - beam.y) ** 2
    return np.exp(-r2 / (2.0 * beam.sigma_x ** 2)) * window(angular_distance(theta_m, beam.theta) / beam.sigma_theta)


def beam_time(beam, t):
    """Temporal factor T(t - tau) of eq. (RTEsources2): a Gaussian, or the
    window w(|t - t_s| / sigma_t) of eq. (sourcelab)."""
    s = t - beam.tau - beam.t0
    if getattr(beam, "profile", "gauss") == "window":
        return window(s / beam.sigma_t)
    return np.exp(-(s ** 2) / (2.0 * beam.sigma_t ** 2))


# ------------------------------------------------------------------ detectors

def detector_tables(spec, xs, ys):
    """Per wall: (weights [Nd, nodes on wall], kappa [M]) so that
    G_j = sum_w weights_w[j] . (u_w @ kappa_w)  (eq. OpMed, discretised)."""
    M = spec.M
    out = []
    for w in walls(spec.Nx, spec.Ny, spec.dx, spec.dy):
        kappa = np.zeros(M)
        for m in range(M):
            if w.dot_sign(m, M) > 0:
                dot = w.dot(m, M)
                kappa[m] = (2.0 * math.pi / M) * (1.0 - fresnel(abs(dot), spec.n_in, spec.n_out)) * dot
        xb = xs[w.is_]
        yb = ys[w.js]
        omega = np.ones(len(w.js))
        omega[0] = omega[-1] = 0.5
        wts = np.zeros((len(spec.detectors), len(w.js)))
        for jd, det in enumerate(spec.detectors):
            dist = np.hypot(xb - det.x, yb - det.y)
            wts[jd] = omega * w.ds * window(dist / det.sigma_d)
        out.append((w, wts, kappa))
    return out
