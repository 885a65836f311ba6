"""Pins of the oracle's scattering, Fresnel, quadrature, window and boundary
map against closed forms and the paper's printed values."""
import math

import numpy as np
import pytest
from scipy.special import i0

from oracle import physics
from tests.golden.values import paper_values

PV = paper_values()


def test_k_phi_trapezoid_matches_paper_and_closed_form():
    # Sec. 5: k_Phi = int exp(-cos^2) dtheta = 4.052876133898710; the DOM
    # trapezoid rule (Sec. 4.1) is spectrally accurate for it
    closed = 2 * math.pi * math.exp(-0.5) * i0(0.5)
    assert abs(closed - PV["k_phi"]) < 1e-14
    errs = []
    for M in (8, 12, 16, 32, 64):
        th, _, _ = physics.ordinates(M)
        errs.append(abs(physics.scalar_flux(np.exp(-np.cos(th) ** 2)[None, :])[0] - PV["k_phi"]))
    # spectral convergence, then round-off
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-8
    assert errs[3] < 4e-15 * PV["k_phi"] and errs[4] < 4e-15 * PV["k_phi"]


@pytest.mark.parametrize("M,g", [(8, 0.5), (16, 0.8), (32, 0.9), (64, 0.95)])
def test_hg_matrix_is_stochastic_symmetric_circulant(M, g):
    W = physics.hg_matrix(M, g, 1.5)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-14)
    assert np.array_equal(W, W.T)
    assert np.allclose(np.roll(np.roll(W, 1, 0), 1, 1), W)
    assert np.argmax(W[3]) == 3  # forward peaked for g > 0


def test_hg_isotropic_limit():
    assert np.allclose(physics.hg_matrix(16, 0.0, 1.5), 1.0 / 16, atol=1e-16)


@pytest.mark.parametrize("M,g", [(8, 0.3), (16, 0.8), (32, 0.9)])
def test_hg_exponent_one_has_poisson_kernel_spectrum(M, g):
    # the circle's HG kernel (1-g^2)/(1+g^2-2g cos) = 1 + 2 sum g^k cos(k theta);
    # sampled at M points and normalised, its DFT is (g^n + g^(M-n)) / (1 + g^M)
    W = physics.hg_matrix(M, g, 1.0)
    eig = np.fft.fft(W[0]).real
    n = np.arange(M)
    assert np.allclose(eig, (g ** n + g ** (M - n)) / (1 + g ** M), atol=1e-13)


def test_fresnel_closed_forms():
    n = 1.4
    assert abs(physics.fresnel(1.0, n, 1.0) - ((n - 1) / (n + 1)) ** 2) < 1e-15
    crit = math.asin(1 / n)
    assert physics.fresnel(math.cos(crit + 1e-6), n, 1.0) == 1.0
    assert physics.fresnel(math.cos(crit - 1e-3), n, 1.0) < 1.0
    assert physics.fresnel(0.3, 1.2, 1.2) == 0.0
    assert physics.fresnel(0.0, n, 1.0) == 1.0  # grazing


@pytest.mark.parametrize("cos_i", [0.999, 0.9, 0.8, 0.75, 0.71])
def test_fresnel_energy_balance(cos_i):
    # R + T = 1 with T from the transmission amplitudes of each polarisation
    n1, n2 = 1.4, 1.0
    R = physics.fresnel(cos_i, n1, n2)
    sin_t = n1 / n2 * math.sqrt(1 - cos_i ** 2)
    cos_t = math.sqrt(1 - sin_t ** 2)
    ts = 2 * n1 * cos_i / (n1 * cos_i + n2 * cos_t)
    tp = 2 * n1 * cos_i / (n2 * cos_i + n1 * cos_t)
    fac = (n2 * cos_t) / (n1 * cos_i)
    T = 0.5 * fac * (ts ** 2 + tp ** 2)
    assert abs(R + T - 1.0) < 1e-14


def test_window_function():
    assert physics.window(0.0) == 1.0
    assert physics.window(1.0) == 0.0 and physics.window(-1.3) == 0.0
    v = np.linspace(-0.99, 0.99, 41)
    assert np.allclose(physics.window(v), physics.window(-v))
    assert np.all(np.diff(physics.window(np.linspace(0, 0.999, 50))) <= 0)
    # continuity at 0 and flatness at 1
    assert abs(physics.window(1e-3) - 1.0) < 1e-12
    assert physics.window(0.95) < 1e-6 and physics.window(0.99) < 1e-30


@pytest.mark.parametrize("M", [8, 12, 16, 32])
def test_reflection_and_incoming_classification(M):
    W4 = physics.walls(4, 4, 0.1, 0.1)
    for w in W4:
        for m in range(M):
            r = w.reflect(m, M)
            assert w.reflect(r, M) == m                       # R o R = id
            assert w.dot_sign(r, M) == -w.dot_sign(m, M)      # incoming <-> outgoing
            assert abs(w.dot(r, M) + w.dot(m, M)) < 1e-14
            exact = w.dot(m, M)
            if w.dot_sign(m, M) == 0:
                assert abs(exact) < 1e-14
            else:
                assert np.sign(exact) == w.dot_sign(m, M)


def test_boundary_entries_counts_and_corner_rule():
    M, N = 16, 6
    j, i, m, sa, ca, sb, cb = physics.boundary_conditions(N, N, M, 0.1, 0.1, 1.4, 1.0)
    # each edge (non-corner) node has exactly the M/2 - 1 strictly incoming ordinates
    edge = (j == 0) & (i > 0) & (i < N)
    assert np.sum(edge) == (N - 1) * (M // 2 - 1)
    # corner (0,0): incoming through x=xmin (cos>0) or y=ymin (sin>0)
    c0 = (j == 0) & (i == 0)
    ms = sorted(m[c0].tolist())
    expect = sorted(k for k in range(M) if physics.cos_sign(k, M) > 0 or physics.sin_sign(k, M) > 0)
    assert ms == expect
    # the diagonal ordinate averages both walls (M % 8 == 0 here)
    diag = c0 & (m == M // 8)
    assert np.sum(diag) == 1 and cb[diag][0] > 0
    # all other corner entries use one wall only
    assert np.all(cb[c0 & (m != M // 8)] == 0)


def test_beam_profile():
    class B:  # minimal beam record
        x, y, theta, sigma_x, sigma_theta, tau, t0, sigma_t = 1.0, 0.0, math.pi / 2, 0.3, math.pi / 4, 5.0, 60.0, 20.0
    th = np.array([math.pi / 2, math.pi / 2 + math.pi / 4, 0.0])
    v = physics.beam_spatial_angular(B, np.array([1.0, 1.0, 1.0]), np.zeros(3), th)
    assert v[0] == 1.0 and v[1] == 0.0 and v[2] == 0.0
    assert physics.beam_time(B, 65.0) == 1.0
    assert abs(physics.beam_time(B, 85.0) - math.exp(-0.5)) < 1e-15
