"""Oracle: the manufactured-solution problem of Sec. 5 (eqs. RTEdisp,
RTEmansol) converges as the paper reports (Fig. 4): fourth order in dt (AB4
with an exact start-up), spectrally in the number of ordinates, and at high
order in h.  A wrong sign or factor in the manufactured source, a wrong
inflow time or a wrong history stalls the error at O(1) or at first order.
Also: the separable source of the library's input helper equals the
oracle's direct formula on the grid."""
import math

import numpy as np

import workloads as W
from oracle.mms import mms_forward, source, u_exact
from oracle.solver import Oracle
from paper_2202_09421_amd.mms import manufactured_inputs

A, B = 0.35, 20.0


def _spec(N, M, dt, T=0.5, L=3.0):
    K = int(round(T / dt))
    sp = W.small_problem(N=N, M=M, K=K, L=L, g=0.0, n_in=1.0, dt=dt, heterogeneous=False, a0=A, b0=B)
    return sp.with_(n_out=1.0)


def _err(N, M, dt):
    return mms_forward(Oracle(_spec(N, M, dt)), A, B)[1]


def test_mms_time_order_four():
    e = [_err(64, 32, dt) for dt in (0.04, 0.02, 0.01)]
    for e0, e1 in zip(e, e[1:]):
        assert 12.0 < e0 / e1 < 20.0, e       # 2^4 = 16


def test_mms_angular_spectral():
    e = [_err(48, M, 0.002) for M in (4, 8, 12)]
    assert e[0] > 100 * e[1] > 100 * 100 * e[2] / 2, e
    assert e[2] < 1e-5


def test_mms_space_high_order():
    e = [_err(N, 32, 0.002) for N in (32, 64)]
    assert e[0] / e[1] > 8.0, e               # order >= 3
    assert e[1] < 3e-7


def test_library_separable_inputs_match_oracle_formula():
    sp = _spec(20, 12, 0.01, T=0.05)
    o = Oracle(sp)
    u0, u_hist, src, inflow = manufactured_inputs(sp, A, B)
    X, Y, Th = src
    for n in (-3, 0, 2, sp.K):
        row = n + 3
        q_sep = np.einsum("kj,ki,km->jim", Y[:, row], X[:, row], Th)
        q_dir = source(o, n * sp.dt, A, B)
        assert np.abs(q_sep - q_dir).max() <= 1e-12 * np.abs(q_dir).max()
        u_sep = np.einsum("kj,ki,km->jim", inflow[1][:, row], inflow[0][:, row], inflow[2])
        assert np.abs(u_sep - u_exact(o, n * sp.dt)).max() <= 1e-15
    assert np.abs(u0[0] - u_exact(o, 0.0)).max() <= 1e-15
    for k in (1, 2, 3):
        assert np.abs(u_hist[k - 1, 0] - u_exact(o, -k * sp.dt)).max() <= 1e-15
