"""AB4 forward solve, misfit and exact discrete adjoint (oracle side).

Forward (Sec. 4.2 eq. RTEAB4, Sec. 4.1 semi-discrete system, Algorithm 1):
for every generalised source q_i (Sec. 3.1) and every step n = 0..K-1,

    L^n    = b (W u^n) - (a + b) u^n - xi_m D_x u^n - eta_m D_y u^n
    u~     = u^n + c dt (chi_0 L^n + chi_1 L^{n-1} + chi_2 L^{n-2} + chi_3 L^{n-3})
    u^{n+1}= BC(u~, t_{n+1})                        (strong overwrite on Gamma_-)
    G^{n+1}= detector readout of u^{n+1}            (eq. OpMed)

with u^0 = 0 and zero history (the paper sets the first time levels to zero)
and t_n = n dt.  chi = (55, -59, 37, -9)/24: the standard fourth-order
Adams-Bashforth weights; the printed chi_0 = 55/44 is read as 55/24 since the
weights of a consistent method sum to one (chi_3 = -9/24 = -3/8 as printed).

Misfit (eqs. FObj, FObjpr): J = 1/2 dt sum_i sum_j sum_{n=1..K} (G^n_{ij} - G~^n_{ij})^2.

Adjoint: the exact transpose of the discrete forward map (the discrete image
of the adjoint problem eq. AdjointProblem: reverse time, final condition zero,
detector misfit entering on Gamma_+, Fresnel reflection transposed).  With
v^k = P^T ubar^k (P the linear part of BC) and v^k = 0 for k > K:

    w^n    = sum_l chi_l v^{n+1+l}
    ubar^n = D_e^T Gbar^n + v^{n+1} + c dt L^T(w^n)
    L^T(w) = b (W^T w) - (a + b) w - D_x^T(xi w) - D_y^T(eta w)
    dJ/da  = -c dt sum_n sum_m u^n_m w^n_m       (discrete eq. FDwin22)
    dJ/db  =  c dt sum_n sum_m u^n_m ((W^T w^n)_m - w^n_m)

for n = K..1, where Gbar = dJ/dG = dt (G - G~).  The gradient is with respect
to the nodal values a_ij, b_ij (what finite differences measure).
"""
from __future__ import annotations

import numpy as np

from . import physics
from .fc import FCLine

CHI = np.array([55.0, -59.0, 37.0, -9.0]) / 24.0


class Oracle:
    """dense_derivative=True applies the same FC operators through their dense
    n x n matrices instead of the FFT: identical mathematics, different rounding
    order.  Tests use the pair to measure the rounding floor of a quantity."""

    def __init__(self, spec, dense_derivative=False):
        self.spec = s = spec
        if s.M % 2:
            raise ValueError("M must be even")
        self.nx, self.ny, self.M = s.Nx + 1, s.Ny + 1, s.M
        self.theta, self.xi, self.eta = physics.ordinates(s.M)
        self.W = physics.hg_matrix(s.M, s.g, s.hg_exponent)
        self.Dx = FCLine(self.nx, s.dx, s.fc_d, s.fc_C, s.filt_alpha, s.filt_beta)
        self.Dy = FCLine(self.ny, s.dy, s.fc_d, s.fc_C, s.filt_alpha, s.filt_beta)
        self.xs = s.xmin + s.dx * np.arange(self.nx)
        self.ys = s.ymin + s.dy * np.arange(self.ny)
        (self.bj, self.bi, self.bm, self.src_a, self.coef_a,
         self.src_b, self.coef_b) = physics.boundary_conditions(s.Nx, s.Ny, s.M, s.dx, s.dy, s.n_in, s.n_out)
        # beams of each generalised source, with their spatial*angular factor on the BC entries
        self.groups = [[bm for bm in s.beams if bm.group == q] for q in range(s.Nq)]
        self.beam_sa = [[physics.beam_spatial_angular(bm, self.xs[self.bi], self.ys[self.bj], self.theta[self.bm])
                         for bm in grp] for grp in self.groups]
        self.det = physics.detector_tables(s, self.xs, self.ys)
        self.inflow = None  # optional callable t -> values on the BC entries
        if dense_derivative:
            for op in (self.Dx, self.Dy):
                Dm = np.ascontiguousarray(op.dense())   # contiguous: the product runs in BLAS
                op.derivative = (lambda D: lambda g, axis=-1: np.moveaxis(np.moveaxis(g, axis, -1) @ D.T, -1, axis))(Dm)
                op.derivative_T = (lambda D: lambda y, axis=-1: np.moveaxis(np.moveaxis(y, axis, -1) @ D, -1, axis))(Dm)

    # ---------------------------------------------------------------- pieces
    def L(self, u, a, b):
        """RHS operator (Algorithm 1 lines 7-15)."""
        dudx = self.Dx.derivative(u, axis=1)
        dudy = self.Dy.derivative(u, axis=0)
        scat = u @ self.W.T
        return b[..., None] * scat - (a + b)[..., None] * u - self.xi * dudx - self.eta * dudy

    def L_T(self, w, a, b):
        scat = w @ self.W
        return (b[..., None] * scat - (a + b)[..., None] * w
                - self.Dx.derivative_T(self.xi * w, axis=1) - self.Dy.derivative_T(self.eta * w, axis=0))

    def source(self, q, t):
        if self.inflow is not None:          # general inflow data (tests only)
            return self.inflow(t)
        val = np.zeros(len(self.bm))
        for bm, sa in zip(self.groups[q], self.beam_sa[q]):
            val += sa * physics.beam_time(bm, t)
        return val

    def apply_bc(self, ut, q, t):
        u = ut.copy()
        u[self.bj, self.bi, self.bm] = (self.coef_a * ut[self.bj, self.bi, self.src_a]
                                        + self.coef_b * ut[self.bj, self.bi, self.src_b]
                                        + self.source(q, t))
        return u

    def apply_bc_T(self, ubar):
        v = ubar.copy()
        tgt = ubar[self.bj, self.bi, self.bm].copy()
        v[self.bj, self.bi, self.bm] = 0.0
        np.add.at(v, (self.bj, self.bi, self.src_a), self.coef_a * tgt)
        np.add.at(v, (self.bj, self.bi, self.src_b), self.coef_b * tgt)
        return v

    def detect(self, u):
        G = np.zeros(len(self.spec.detectors))
        for (w, wts, kappa) in self.det:
            G += wts @ (u[w.js, w.is_, :] @ kappa)
        return G

    def detect_T(self, gbar, out):
        for (w, wts, kappa) in self.det:
            out[w.js, w.is_, :] += np.outer(gbar @ wts, kappa)
        return out

    # ---------------------------------------------------------------- solves
    def forward(self, mu_a=None, mu_s=None, keep_states=False, K=None, q_list=None, u0=None):
        """Returns G [Nq, Nd, K] (G[q, j, n-1] = G_j^n), u^K [Nq, ny, nx, M] and,
        if asked, the states u^0..u^K per source.  u0 (tests only) replaces the
        vanishing initial state; the AB4 history still starts at zero."""
        s = self.spec
        a = s.mu_a if mu_a is None else mu_a
        b = s.mu_s if mu_s is None else mu_s
        K = s.K if K is None else K
        qs = range(s.Nq) if q_list is None else q_list
        cdt = s.c * s.dt
        G = np.zeros((s.Nq, len(s.detectors), K))
        uK = np.zeros((s.Nq, self.ny, self.nx, self.M))
        states = {}
        for q in qs:
            u = np.zeros((self.ny, self.nx, self.M)) if u0 is None else np.array(u0, dtype=np.float64)
            hist = [np.zeros_like(u) for _ in range(3)]
            traj = [u] if keep_states else None
            for n in range(K):
                Ln = self.L(u, a, b)
                ut = u + cdt * (CHI[0] * Ln + CHI[1] * hist[0] + CHI[2] * hist[1] + CHI[3] * hist[2])
                u = self.apply_bc(ut, q, (n + 1) * s.dt)
                hist = [Ln, hist[0], hist[1]]
                G[q, :, n] = self.detect(u)
                if keep_states:
                    traj.append(u)
            uK[q] = u
            if keep_states:
                states[q] = traj
        return G, uK, states

    def misfit(self, G, Gmeas):
        return 0.5 * self.spec.dt * float(np.sum((G - Gmeas) ** 2))

    def adjoint(self, Gbar, states, mu_a=None, mu_s=None, want_u0bar=False):
        """Exact transpose of the forward map.  Gbar = dJ/dG [Nq, Nd, K].
        Returns dJ/da, dJ/db [ny, nx] summed over the sources (and, if asked,
        dJ/du^0 per source, used by the dot-product test)."""
        s = self.spec
        a = s.mu_a if mu_a is None else mu_a
        b = s.mu_s if mu_s is None else mu_s
        K = Gbar.shape[2]
        cdt = s.c * s.dt
        ga = np.zeros((self.ny, self.nx))
        gb = np.zeros((self.ny, self.nx))
        u0bar = {}
        for q, traj in states.items():
            zero = np.zeros((self.ny, self.nx, self.M))
            v = {}  # v^k for k = n+1..n+4

            def getv(k):
                return v.get(k, zero)

            for n in range(K, -1, -1):
                w = sum(CHI[l] * getv(n + 1 + l) for l in range(4))
                un = traj[n]
                ga += -cdt * np.sum(un * w, axis=-1)
                gb += cdt * np.sum(un * (w @ self.W - w), axis=-1)
                if n == 0:   # u^0 is data: no detector reading, no boundary overwrite
                    if want_u0bar:
                        u0bar[q] = getv(1) + cdt * self.L_T(w, a, b)
                    break
                ubar = self.detect_T(Gbar[q, :, n - 1], getv(n + 1).copy())
                ubar += cdt * self.L_T(w, a, b)
                v[n] = self.apply_bc_T(ubar)
                v.pop(n + 4, None)
        if want_u0bar:
            return ga, gb, u0bar
        return ga, gb

    def gradient(self, Gmeas, mu_a=None, mu_s=None):
        """J and its gradients with respect to the nodal a and b."""
        G, _, states = self.forward(mu_a, mu_s, keep_states=True)
        J = self.misfit(G, Gmeas)
        ga, gb = self.adjoint(self.spec.dt * (G - Gmeas), states, mu_a, mu_s)
        return J, ga, gb, G
