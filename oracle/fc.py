"""FC-Gram continuation and filtered spectral derivative (oracle side).

Sec. 4.3.  For a line g = (g_1..g_n) of nodal values with spacing h:

1. the last d values are projected on the Gram basis, c_R = Q^T g[n-d:n], and
   the first d values (read outward, i.e. reversed) give c_L = Q^T rev(g[0:d]);
2. the precomputed blends give the right continuation A c_R (C values leaving
   g_n) and the left continuation A c_L (C values approaching g_1 when read
   backwards);
3. both are padded with E zeros to C + E values, the right one at its start and
   the left one at its end (the paper's g_r = [g~_r; 0], g_l = [0; g~_l]);
4. g_c = [g; g_l + g_r] has N_p = n + C + E entries, E being the smallest
   count that makes N_p a product of primes <= 5.

eq. (RTEFCSum) expands g_c in a Fourier series of period N_p h (reading: the
printed "(N_p - 1) h" would make the derivative inconsistent at first order),
eq. (FFilter) multiplies the coefficients by exp(-alpha |2k/N_p|^(2 beta))
with alpha = 2, beta = 55, and eq. (RTEFCSumder) differentiates term by term.
For even N_p the k = N_p/2 coefficient of the derivative is set to zero
(reading: the printed sum runs over both ends, which would make the output
complex).  The derivative at the n grid nodes is the first n entries.

The FFT is numpy's (a library primitive); everything else is written out.
set_fft_workers(n) switches it to scipy's (the same pocketfft algorithm) with
n threads, for timing the oracle on every host core.
"""
from __future__ import annotations

import numpy as np

from .fc_gram import blend_table

_FFT_WORKERS = None


def set_fft_workers(n):
    """None: numpy.fft (one thread).  n >= 1: scipy.fft with n worker threads."""
    global _FFT_WORKERS
    _FFT_WORKERS = n


def _fft(x):
    if _FFT_WORKERS is None:
        return np.fft.fft(x, axis=-1)
    import scipy.fft
    return scipy.fft.fft(x, axis=-1, workers=_FFT_WORKERS)


def _ifft(x):
    if _FFT_WORKERS is None:
        return np.fft.ifft(x, axis=-1)
    import scipy.fft
    return scipy.fft.ifft(x, axis=-1, workers=_FFT_WORKERS)


def is_5smooth(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def extra_points(n: int, C: int) -> int:
    """E of step 3: the smallest E >= 0 with n + C + E 5-smooth."""
    E = 0
    while not is_5smooth(n + C + E):
        E += 1
    return E


def multiplier(Np: int, h: float, alpha: float = 2.0, beta: float = 55.0) -> np.ndarray:
    """Filtered derivative factor per DFT index k (eqs. FFilter, RTEFCSumder)."""
    k = np.arange(Np)
    kappa = np.where(k <= Np // 2, k, k - Np).astype(np.float64)
    lam = 1j * (2.0 * np.pi * kappa / (Np * h)) * np.exp(-alpha * np.abs(2.0 * kappa / Np) ** (2.0 * beta))
    if Np % 2 == 0:
        lam[Np // 2] = 0.0
    return lam


class FCLine:
    """The FC derivative operator for lines of n nodes and spacing h."""

    def __init__(self, n: int, h: float, d: int = 5, C: int = 25, alpha: float = 2.0, beta: float = 55.0):
        if n < 2 * d:
            raise ValueError("a line needs at least 2d nodes")
        self.n, self.h, self.d, self.C = n, h, d, C
        self.Q, self.A = blend_table(d, C)
        self.E = extra_points(n, C)
        self.Np = n + C + self.E
        self.lam = multiplier(self.Np, h, alpha, beta)
        # Step 1+2 as one matrix from the d matching values to the C blend values
        # (the right end; the left end is its mirror image).
        self.B = self.Q @ self.A.T  # [d, C]: ext_R = g[n-d:n] @ B

    # -- steps 1-4: the continued vector g_c (last axis is the line)
    def continue_line(self, g: np.ndarray) -> np.ndarray:
        n, d, C, E = self.n, self.d, self.C, self.E
        ext = np.zeros(g.shape[:-1] + (C + E,), dtype=g.dtype)
        ext[..., :C] += g[..., n - d:] @ self.B                 # g_r = [g~_r ; 0_E]
        left = g[..., d - 1::-1] @ self.B                       # blend read outward from g_1
        ext[..., E:] += left[..., ::-1]                         # g_l = [0_E ; g~_l]
        return np.concatenate([g, ext], axis=-1)

    def periodic_derivative(self, gc: np.ndarray) -> np.ndarray:
        return _ifft(self.lam * _fft(gc)).real

    def derivative(self, g: np.ndarray, axis: int = -1) -> np.ndarray:
        g = np.moveaxis(np.asarray(g, dtype=np.float64), axis, -1)
        out = self.periodic_derivative(self.continue_line(g))[..., : self.n]
        return np.moveaxis(out, -1, axis)

    # -- the exact transpose of `derivative` (needed by the discrete adjoint)
    def derivative_T(self, y: np.ndarray, axis: int = -1) -> np.ndarray:
        y = np.moveaxis(np.asarray(y, dtype=np.float64), axis, -1)
        n, d, C, E, Np = self.n, self.d, self.C, self.E, self.Np
        z = np.zeros(y.shape[:-1] + (Np,))
        z[..., :n] = y                                            # transpose of "first n entries"
        # transpose of the real circulant: conjugate multiplier
        z = _ifft(np.conj(self.lam) * _fft(z)).real
        g = z[..., :n].copy()                                     # transpose of [g; ext]
        zext = z[..., n:]
        g[..., n - d:] += zext[..., :C] @ self.B.T                # transpose of the right blend
        g[..., d - 1::-1] += zext[..., E:][..., ::-1] @ self.B.T  # transpose of the left blend
        return np.moveaxis(g, -1, axis)

    def dense(self) -> np.ndarray:
        """The n x n matrix of the operator (for tests on small n)."""
        return self.derivative(np.eye(self.n), axis=0)
