"""GPU: plans whose state arrays exceed 64 MiB per combination chunk stream
them with the non-temporal hint (node passes, and the line passes' stores
where it pays); smaller plans use ordinary loads and stores.  The hint only
changes cache placement, so a plan on either side of the threshold must give
the same gradient bit for bit.  The chunked and unchunked runs of one problem
compute every element by the same arithmetic, which makes them the pair to
compare: at 257 x 257 nodes, 4 combinations in one chunk are above the
threshold and one combination per chunk is below it.  (J sums over chunks,
so it agrees to rounding only.)"""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

THRESHOLD = 64 << 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rte():
    from paper_2202_09421_amd import rte as R
    R.lib()
    return R


def _spec(M):
    beams = []
    for k, (x, y) in enumerate([(0.5, 0.0), (1.0, 0.5), (0.5, 1.0), (0.0, 0.4)]):
        b = W.beam_at(x, y, 0, 1, 0, 1, sigma_t=2.0, t0=1.0, sigma_x=0.1, tau=0.3 * k)
        b.group = k
        beams.append(b)
    return W.small_problem(N=256, M=M, K=10, seed=41, n_in=1.4, n_det=8).with_(beams=beams)


def _state_bytes(spec, dtype, chunk):
    # one state array of a chunk: [chunk][M / 4 groups][ny][nxp][4 slots], rows
    # padded to 128 bytes per group (4 FP64 or 8 FP32 nodes), plus one such
    # unit when the row pitch is a multiple of 2 KB
    es = 8 if dtype == torch.float64 else 4
    align = 128 // (4 * es)
    nx, ny = spec.Nx + 1, spec.Ny + 1
    nxp = -(-nx // align) * align
    if (nxp * 4 * es) % 2048 == 0:
        nxp += align
    return chunk * spec.M * ny * nxp * es


@pytest.mark.parametrize("dtype,M", [(torch.float64, 32), (torch.float32, 64)])
def test_streamed_and_cached_plans_bitwise_equal(rte, dtype, M):
    spec = _spec(M)
    assert _state_bytes(spec, dtype, 4) > THRESHOLD > _state_bytes(spec, dtype, 1)
    rng = np.random.default_rng(3)
    Gm = 1e-4 * rng.standard_normal((4, len(spec.detectors), spec.K))
    outs = []
    for chunk in (4, 1):
        say("%s M=%d chunk %d: state array %.1f MiB" % (dtype, M, chunk, _state_bytes(spec, dtype, chunk) / 2**20))
        pl = rte.Plan(spec, dtype, combo_chunk=chunk, ckpt_every=4)
        J, ga, gb, G = pl.gradient(spec.mu_a, spec.mu_s, Gm)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy().copy() for t in (J, ga, gb, G)])
        pl.close()
    assert np.abs(outs[0][3]).max() > 0
    # J sums the misfit chunk by chunk, so its rounding follows the chunking;
    # the traces and both gradient maps are elementwise and must be equal
    J4, J1 = float(outs[0][0].ravel()[0]), float(outs[1][0].ravel()[0])
    say("J rel diff %.1e" % (abs(J4 - J1) / abs(J1)))
    assert abs(J4 - J1) <= 1e-14 * abs(J1)
    for k in (1, 2, 3):
        assert np.array_equal(outs[0][k], outs[1][k]), k
