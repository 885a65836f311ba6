"""Oracle expectations for the full-size GPU parity tests (run on a CPU):

    python -m tests.golden.make_fullsize [name ...]

Each case is a full-size plan shape of the benchmark workloads with the
gradient evaluated through the whole path (forward, misfit, adjoint) over a
K short enough for the FP64 NumPy oracle, and the pulses moved to the start
so that the detectors are lit:
  * bench257: 257 x 257 nodes, 32 ordinates, N_p = 288 lines, one beam,
    32 detectors, K = 300 (the FP64 gradient workload's plan);
  * mss513: 513 x 513 nodes, 64 ordinates, N_p = 540 lines, two MSS
    combinations of two beams each, 64 detectors, K = 15 (the batched MSS
    workload's plan).
The measured traces are the oracle's forward traces of the medium with
inclusions times (1 + 0.1 xi); the gradient is taken at the homogeneous
background, as in the paper's inversions.  Stored: the measured traces and
the oracle's G, J, dJ/dmu_a, dJ/dmu_s, plus the rounding floors of each
(the oracle's FFT path against its dense-matrix path, and the effect on J
and the gradients of perturbations of G at G's floor).  Only oracle/ and
workloads/ are called.
"""
from __future__ import annotations

import dataclasses
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.solver import Oracle  # noqa: E402

CASES = ("bench257", "mss513")


def fullsize_case(name):
    """(spec at the background medium, true medium (a, b), run settings)."""
    if name == "bench257":
        full = W.config(1)
        spec = full.with_(K=300, beams=[dataclasses.replace(b, t0=5.0) for b in full.beams])
        settings = dict(ckpt_every=0, combo_chunk=0)
    elif name == "mss513":
        full = W.config(2)
        keep = {0: 0, 5: 1}
        beams = [dataclasses.replace(b, group=keep[b.group], tau=0.0, t0=0.0) for b in full.beams if b.group in keep]
        spec = full.with_(K=15, beams=beams)
        settings = dict(ckpt_every=4, combo_chunk=1)
    else:
        raise ValueError(name)
    true_medium = (spec.mu_a.copy(), spec.mu_s.copy())
    bg = spec.with_(mu_a=np.full_like(spec.mu_a, 0.2), mu_s=np.full_like(spec.mu_s, 50.0))
    return bg, true_medium, settings


def path(name):
    return os.path.join(HERE, "fullsize_%s.npz" % name)


def rel(a, b):
    den = np.linalg.norm(np.ravel(b))
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / (den if den > 0 else 1.0))


def make(name):
    spec, (a_true, b_true), _ = fullsize_case(name)
    o = Oracle(spec)
    G_true = o.forward(a_true, b_true)[0]
    Gm = G_true * W.measured_noise(7, G_true.shape)
    G, _, st = o.forward(keep_states=True)
    J = o.misfit(G, Gm)
    ga, gb = o.adjoint(spec.dt * (G - Gm), st)
    print(name, "oracle gradient done", flush=True)
    Jd, gad, gbd, Gd = Oracle(spec, dense_derivative=True).gradient(Gm)
    floor = dict(G=rel(Gd, G), J=abs(Jd - J) / abs(J), ga=rel(gad, ga), gb=rel(gbd, gb))
    for trial in range(3):
        dG = np.random.default_rng(1000 + trial).standard_normal(G.shape)
        dG *= max(floor["G"], 1e-16) * np.linalg.norm(G) / np.linalg.norm(dG)
        gap, gbp = o.adjoint(spec.dt * (G + dG - Gm), st)
        floor["J"] = max(floor["J"], abs(o.misfit(G + dG, Gm) - J) / abs(J))
        floor["ga"] = max(floor["ga"], rel(gap, ga))
        floor["gb"] = max(floor["gb"], rel(gbp, gb))
    print(name, "floors", floor, flush=True)
    np.savez_compressed(path(name), Gm=Gm, G=G, J=np.array(J), ga=ga, gb=gb,
                        floor=np.array([floor[k] for k in ("G", "J", "ga", "gb")]))


if __name__ == "__main__":
    from oracle import fc as _ofc
    _ofc.set_fft_workers(os.cpu_count() or 1)   # the same FFT on every core
    for nm in (sys.argv[1:] or CASES):
        make(nm)
