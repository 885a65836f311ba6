"""Pins of the oracle's FC-Gram derivative against what the paper and the
mathematics fix (Sec. 4.3)."""
import numpy as np
import pytest

from oracle.fc import FCLine, extra_points, multiplier, is_5smooth
from oracle.fc_gram import blend_table
from tests.golden.values import paper_values

PV = paper_values()


def test_extra_points_reproduce_paper_example():
    # Sec. 4.3: N=60 intervals (61 nodes), C=25 -> E=4, N_p=90 = 2*3*3*5
    n = PV["fc_example_N"] + 1
    E = extra_points(n, PV["fc_example_C"])
    assert E == PV["fc_example_E"]
    assert n + PV["fc_example_C"] + E == PV["fc_example_Np"]


@pytest.mark.parametrize("n,Np", [(65, 90), (129, 160), (257, 288), (513, 540), (1025, 1080)])
def test_extension_sizes_are_smallest_5smooth(n, Np):
    E = extra_points(n, 25)
    assert n + 25 + E == Np
    assert all(not is_5smooth(k) for k in range(n + 25, Np))


def test_gram_basis_orthonormal_and_polynomial():
    Q, A = blend_table(5, 25)
    assert np.allclose(Q.T @ Q, np.eye(5), atol=1e-14)
    s = np.arange(5.0)
    for j in range(5):
        # column j is a polynomial of exact degree j with positive leading coefficient
        coef = np.polyfit(s, Q[:, j], j)
        assert np.allclose(np.polyval(coef, s), Q[:, j], atol=1e-13)
        assert coef[0] > 0


def test_blend_decays_to_zero():
    # the blends leave the matching values and reach ~0 at the end of the C points
    Q, A = blend_table(5, 25)
    assert A.shape == (25, 5)
    assert np.abs(A[-1]).max() < 1e-4
    assert np.abs(A[0]).max() > 1e-2


def _conv(f, df, a, b, Ns):
    errs = []
    for N in Ns:
        x = np.linspace(a, b, N + 1)
        op = FCLine(N + 1, (b - a) / N)
        errs.append(np.max(np.abs(op.derivative(f(x)) - df(x))) / np.max(np.abs(df(x))))
    return np.array(errs)


def test_high_order_on_paper_example_function():
    # g(x) = 12 + x^2 - exp(x/3) on [0, 6] (Sec. 4.3, Fig. 2)
    errs = _conv(lambda x: 12 + x ** 2 - np.exp(x / 3), lambda x: 2 * x - np.exp(x / 3) / 3,
                 0.0, 6.0, [16, 32, 64, 128])
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 3.5), (errs, orders)
    assert errs[-1] < 1e-8
    # the paper's own N=60 case is already accurate
    assert _conv(lambda x: 12 + x ** 2 - np.exp(x / 3), lambda x: 2 * x - np.exp(x / 3) / 3, 0, 6, [60])[0] < 1e-6


def test_high_order_on_oscillatory_function():
    errs = _conv(lambda x: np.sin(3 * x + 1), lambda x: 3 * np.cos(3 * x + 1), 0.0, 2.0, [32, 64, 128, 256])
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 3.5), (errs, orders)


def test_low_degree_polynomials_nearly_exact():
    x = np.linspace(-1.0, 2.0, 97)
    op = FCLine(97, 3.0 / 96)
    for deg in range(3):
        p = np.poly1d(np.arange(1, deg + 2, dtype=float))
        err = np.max(np.abs(op.derivative(p(x)) - p.deriv()(x)))
        assert err < 1e-7, (deg, err)


def test_reflection_equivariance():
    # reversing a line negates and reverses its derivative iff the left blend
    # is the mirror image of the right blend (step 3 placement)
    rng = np.random.default_rng(0)
    for n in (40, 65, 101):
        g = rng.standard_normal(n)
        op = FCLine(n, 0.1)
        assert np.allclose(op.derivative(g[::-1]), -op.derivative(g)[::-1], atol=1e-10)


def test_period_is_Np_times_h():
    # a Fourier mode of the extended grid is differentiated exactly (filter ~ 1
    # for low modes): this pins the period N_p h of eq. (RTEFCSum)
    op = FCLine(65, 0.03)
    Np, h = op.Np, op.h
    xg = h * np.arange(Np)
    for k in (1, 3, 7):
        gc = np.sin(2 * np.pi * k * xg / (Np * h))
        d = op.periodic_derivative(gc)
        exact = 2 * np.pi * k / (Np * h) * np.cos(2 * np.pi * k * xg / (Np * h))
        assert np.allclose(d, exact, atol=1e-11 * np.abs(exact).max())


def test_filter_and_nyquist():
    lam = multiplier(90, 1.0)
    k = np.arange(90)
    kappa = np.where(k <= 45, k, k - 90)
    assert lam[45] == 0
    # odd, purely imaginary: the periodic operator is real and skew-symmetric
    assert np.all(lam.real == 0)
    assert np.allclose(lam[1:45], -lam[89:45:-1])
    # filter: ~1 for low modes, exp(-2) at |2k/N_p| = 1
    assert np.isclose(lam[10].imag, 2 * np.pi * 10 / 90, rtol=1e-15)
    assert np.isclose(lam[44].imag / (2 * np.pi * 44 / 90), np.exp(-2 * (88 / 90) ** 110), rtol=1e-12)


def test_transpose_matches_dense_matrix():
    for n in (10, 33, 65):
        op = FCLine(n, 0.07)
        D = op.dense()
        DT = op.derivative_T(np.eye(n), axis=0)
        assert np.allclose(DT, D.T, atol=1e-12 * np.abs(D).max())
        rng = np.random.default_rng(n)
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        assert np.isclose(y @ op.derivative(x), x @ op.derivative_T(y), rtol=1e-12)


def test_batched_axes_agree_with_single_lines():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((20, 17, 4))
    opx = FCLine(17, 0.1)
    opy = FCLine(20, 0.2)
    dx = opx.derivative(u, axis=1)
    dy = opy.derivative(u, axis=0)
    assert np.allclose(dx[5, :, 2], opx.derivative(u[5, :, 2]), atol=1e-13)
    assert np.allclose(dy[:, 7, 1], opy.derivative(u[:, 7, 1]), atol=1e-13)
