"""FC-Gram tables for the library (plan-time precomputation, host side).

Sec. 4.3 step 1-2: the d matching values at each line end are projected on
a Gram polynomial basis and every basis polynomial has a precomputed smooth
blend to zero over C points.  The paper cites but does not print the
construction; this library uses the following definition:

  Q[k, j] = P_j(k): polynomials orthonormal over s = 0..d-1 (grid units),
            degree j, positive leading coefficient -- the Q factor of the
            QR factorisation of the Vandermonde matrix [k^j].
  A[p, j] = T_j(d + p), p = 0..C-1, where T_j is the least-squares
            trigonometric polynomial of period 2(d+C) with (d+C)//2 modes
            matching P_j on [0, d-1] and 0 on [d+C, 2d+C-1], both sampled
            20 times per grid spacing.

The least-squares problem (condition ~4e14) is solved by Householder QR in
80-digit arithmetic and rounded to double, so the tables are the exact
values of that definition to the last bit of a double.
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np

_DIGITS = 80
_SAMPLES_PER_H = 20


@functools.lru_cache(maxsize=None)
def fc_tables(d: int = 5, C: int = 25):
    """Return (Q [d, d], A [C, d]) as float64 arrays (row-major)."""
    with mpmath.workdps(_DIGITS):
        V = mpmath.matrix(d, d)
        for k in range(d):
            for j in range(d):
                V[k, j] = mpmath.mpf(k) ** j
        Qm, Rm = mpmath.qr(V)
        for j in range(d):  # sign convention: positive leading coefficients
            if Rm[j, j] < 0:
                for k in range(d):
                    Qm[k, j] = -Qm[k, j]

        period = 2 * (d + C)
        modes = (d + C) // 2

        def basis(s):
            out = [mpmath.mpf(1)]
            for l in range(1, modes + 1):
                a = 2 * mpmath.pi * l * s / period
                out += [mpmath.cos(a), mpmath.sin(a)]
            return out

        step = mpmath.mpf(1) / _SAMPLES_PER_H
        nsamp = (d - 1) * _SAMPLES_PER_H + 1
        match = [k * step for k in range(nsamp)]
        zero = [mpmath.mpf(d + C) + k * step for k in range(nsamp)]
        X = mpmath.matrix([basis(s) for s in match + zero])

        # Lagrange form of each Gram polynomial: P_j(s) = sum_k Q[k, j] l_k(s)
        def lagrange(s):
            vals = []
            for k in range(d):
                v = mpmath.mpf(1)
                for i in range(d):
                    if i != k:
                        v *= (s - i) / mpmath.mpf(k - i)
                vals.append(v)
            return vals

        Lm = [lagrange(s) for s in match]
        ev = mpmath.matrix([basis(mpmath.mpf(d + p)) for p in range(C)])
        A = np.empty((C, d))
        for j in range(d):
            rhs = mpmath.matrix([sum(Qm[k, j] * Lm[t][k] for k in range(d)) for t in range(nsamp)] + [0] * nsamp)
            coef, _res = mpmath.qr_solve(X, rhs)
            vals = ev * coef
            for p in range(C):
                A[p, j] = float(vals[p])
        Q = np.array([[float(Qm[k, j]) for j in range(d)] for k in range(d)])
    return Q, A
