"""FC-Gram blend-to-zero tables (oracle side).

Sec. 4.3 (the four-step continuation): the d matching values at a line end
are projected on a Gram polynomial basis, and each basis polynomial has an
accurately precomputed smooth continuation to zero over C points.  The paper
cites the construction (Albin & Bruno 2011, Amlani & Bruno 2016) but prints
neither the recipe nor the values.  This oracle fixes one reading and writes
it out plainly:

* Gram basis: polynomials P_0..P_{d-1} orthonormal for the discrete inner
  product over the matching points s = 0..d-1 (grid units), built by
  Gram-Schmidt on the monomials 1, s, s^2, ...; leading coefficient > 0.
  Q[k, j] = P_j(k).
* Blend of P_j: the trigonometric polynomial
      T(s) = a_0 + sum_{l=1}^{L} a_l cos(2 pi l s / Lam) + b_l sin(2 pi l s / Lam)
  of period Lam = 2 (d + C) and L = (d + C) // 2 modes that minimises, in
  plain least squares,
      sum_{s in S_match} (T(s) - P_j(s))^2 + sum_{s in S_zero} T(s)^2,
  S_match = {k/20 : 0 <= k <= 20 (d-1)}        (the matching interval [0, d-1]),
  S_zero  = {d + C + k/20 : 0 <= k <= 20 (d-1)} (a zero interval after the C points).
* A[p, j] = T_j(d + p), p = 0..C-1: the C continuation values.

The least-squares matrix has condition ~4e14, so it is solved through the
normal equations in 80-digit arithmetic (mpmath) and rounded to double.

Exact table values are parity unpinned against the paper; what pins them is
the behaviour of the derivative they produce (tests/test_oracle_fc.py).
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

_DPS = 80
_OVERSAMPLE = 20


def _gram_schmidt(d: int):
    """Orthonormal polynomials on s = 0..d-1, returned as their values there."""
    pts = [mp.mpf(k) for k in range(d)]
    basis = []
    for j in range(d):
        v = [p ** j for p in pts]
        for q in basis:
            dot = mp.fsum(v[k] * q[k] for k in range(d))
            v = [v[k] - dot * q[k] for k in range(d)]
        # a second pass keeps the basis orthogonal to working precision
        for q in basis:
            dot = mp.fsum(v[k] * q[k] for k in range(d))
            v = [v[k] - dot * q[k] for k in range(d)]
        nrm = mp.sqrt(mp.fsum(x * x for x in v))
        basis.append([x / nrm for x in v])
    return basis  # basis[j][k] = P_j(k)


def _poly_eval(values, d: int, s):
    """Value at s of the degree-(d-1) polynomial through (k, values[k])."""
    tot = mp.mpf(0)
    for k in range(d):
        lk = mp.mpf(1)
        for i in range(d):
            if i != k:
                lk *= (s - i) / mp.mpf(k - i)
        tot += values[k] * lk
    return tot


@functools.lru_cache(maxsize=None)
def blend_table(d: int = 5, C: int = 25):
    """Return (Q, A): Q d x d Gram values, A C x d continuation values (float64)."""
    with mp.workdps(_DPS):
        Lam = 2 * (d + C)
        L = (d + C) // 2
        s_match = [mp.mpf(k) / _OVERSAMPLE for k in range((d - 1) * _OVERSAMPLE + 1)]
        s_zero = [mp.mpf(d + C) + mp.mpf(k) / _OVERSAMPLE for k in range((d - 1) * _OVERSAMPLE + 1)]

        def trig_row(s):
            row = [mp.mpf(1)]
            for l in range(1, L + 1):
                ang = 2 * mp.pi * l * s / Lam
                row.append(mp.cos(ang))
                row.append(mp.sin(ang))
            return row

        X = mp.matrix([trig_row(s) for s in s_match + s_zero])
        XtX = X.T * X
        basis = _gram_schmidt(d)
        ev = mp.matrix([trig_row(mp.mpf(d + p)) for p in range(C)])
        A = np.zeros((C, d))
        for j in range(d):
            rhs = mp.matrix([_poly_eval(basis[j], d, s) for s in s_match] + [mp.mpf(0)] * len(s_zero))
            coef = mp.lu_solve(XtX, X.T * rhs)
            vals = ev * coef
            A[:, j] = [float(vals[p]) for p in range(C)]
        Q = np.array([[float(basis[j][k]) for j in range(d)] for k in range(d)])
    return Q, A
