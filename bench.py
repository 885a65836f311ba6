#!/usr/bin/env python3
"""Benchmark of the FC-DOM forward + adjoint gradient on one MI355X.

Default workload (the metric's configuration): the batched multiple-
staggered-source problem, 6 x 6 cm, 513 x 513 nodes, 64 ordinates, HG
g = 0.9, Fresnel n = 1.4, background mu_a = 0.2 / mu_s = 50 per cm (three
inclusions in the true medium), 16 beams fired as 8 combinations of two with
seeded delays 0..100 ps, 64 detectors, 6000 AB4 steps, FP64.  One gradient
evaluation: forward of all 8 combinations with checkpoints, misfit against
synthetic measurements (forward on the medium with inclusions, 10 %
multiplicative noise), checkpointed segment replay and exact discrete
adjoint, dJ/dmu_a and dJ/dmu_s.  "batched": combination chunks as large as
HBM allows (every launch covers a whole chunk); "plain": one combination per
launch, one after another.

One benchmark step = one slice of the batched gradient: the gradient's fixed
sequence of operations (rte_gradient_ops) cut into --steps ranges of equal
operation count (rte_gradient_range), so the --steps timed steps are exactly
one whole gradient (bit-identical to one rte_gradient call) and
steps x ms_per_step is its wall time.  Warmup steps run the first --warmup
slices of another gradient.  The plain gradient is timed as one call.

value = cells * ordinates * time steps * combinations / seconds per gradient
(a unit is one node x one ordinate x one step, counted once for the whole
forward + replay + adjoint).  Inputs are resident in HBM before the timed
region.

Prints one JSON line (last line of stdout).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
WORD = {"f64": 8, "f32": 4}

# compulsory words moved per unit (node x ordinate) by one launch of each kernel class
KERNEL_WORDS = {
    "lines_fwd": 4,    # x and y lines: read u twice, write -xi Dx u and -eta Dy u
    "node_fwd": 8,     # read u, X, Y, L^{n-1..n-3}; write u^{n+1}, L^n
    "node_adj": 10,    # read atx, aty, P1^{n+1}, v^{n+2..n+4}, u^n; write v^{n+1}, w^n, P1^n
    "lines_adj": 4,    # x and y lines: read w twice, write Dx^T(xi w) and Dy^T(eta w)
}
PATH_WORDS_STORE_ALL = 12  # algorithmic fwd + adj per unit: 6 + 6 words
PATH_WORDS_REPLAY = 19     # with one-level checkpoint replay: 6 + 6 + 6 + 1 store
# algorithmic words per unit of one launch: a node pass completes one time step
# (forward: read u, L^{n-1..n-3}, write u, L^n; adjoint: read v^{n+1..n+4}, u^n,
# write v^n); the line passes only move intermediates and are charged their
# own compulsory words
ALGO_WORDS = {"node_fwd": 6, "node_adj": 6, "lines_fwd": 4, "lines_adj": 4}

# kernel class -> row label in the committed HBM counter summary
TRAFFIC_ROWS = {
    "lines_fwd": "x and y line derivatives (fwd)", "node_fwd": "node pass (fwd)",
    "node_adj": "node pass (adj)", "lines_adj": "x and y line transposes (adj)",
}
TRAFFIC_FILE = {("mss", "f64"): "profiles/mss_fp64_513x513_M64_chunk4_hbm_traffic.md",
                ("mss", "f32"): "profiles/mss_fp32_513x513_M64_chunk8_hbm_traffic.md"}


def source_hash():
    """sha256 over the kernel sources (.hip and .h files of csrc: file name,
    then bytes, sorted by name); host-only files do not change the traffic."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = glob.glob(os.path.join(ROOT, "paper_2202_09421_amd", "csrc", "*.hip")) + \
        glob.glob(os.path.join(ROOT, "paper_2202_09421_amd", "csrc", "*.h"))
    for f in sorted(files, key=os.path.basename):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, dtype, cls):
    """HBM bytes per launch of kernel class `cls` from the committed
    FETCH_SIZE / WRITE_SIZE summary (already scaled by the copy calibration),
    or None when no summary exists or the kernels changed since it was taken."""
    import re
    name = TRAFFIC_FILE.get((workload, dtype))
    if name is None or not os.path.exists(os.path.join(ROOT, name)):
        return None
    with open(os.path.join(ROOT, name)) as fh:
        text = fh.read()
    m = re.search(r"source-hash ([0-9a-f]{16})", text)
    if m is None or m.group(1) != source_hash():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0].startswith(TRAFFIC_ROWS[cls]):
            rd, wr = float(cells[2]), float(cells[3])
            return {"bytes": (rd + wr) * (1 << 20), "read_MiB": rd, "write_MiB": wr, "source": name}
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(spec, target_s=15.0):
    """Time the FP64 oracle (single thread) on the first steps of the same
    workload: forward + adjoint gradient on the full grid."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.solver import Oracle

    with threadpool_limits(limits=1):
        o = Oracle(spec.with_(K=2))
        t0 = time.perf_counter()
        o.gradient(np.zeros((1, len(spec.detectors), 2)))
        per_step = (time.perf_counter() - t0) / 2
        Ks = int(max(4, min(60, target_s / max(per_step, 1e-3))))
        sample = spec.with_(K=Ks)
        o = Oracle(sample)
        t0 = time.perf_counter()
        o.gradient(np.zeros((1, len(spec.detectors), Ks)))
        dt = time.perf_counter() - t0
    units = (spec.Nx + 1) * (spec.Ny + 1) * spec.M * Ks * spec.Nq
    return {"value": units / dt, "unit": "cell*ordinate*steps/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d steps of the same workload (full 257x257 grid, 32 ordinates), "
                      "forward + adjoint gradient, NumPy FP64, 1 thread, %.1f s" % (Ks, spec.K, dt)}


def mss_comparison(K, dtype_name, log_fn):
    """Multiple-staggered-source workload (8 combinations of 2 delayed beams on
    a 513 x 513 grid, 64 ordinates): the gradient of all combinations in one
    batched plan (every launch covers all 8) against 8 single-combination plans
    solved one after another ("plain"), same kernels, graph replay for both.
    Returns throughputs and the difference of the summed gradients."""
    import dataclasses

    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte

    tdt = torch.float64 if dtype_name == "f64" else torch.float32
    full = W.config(2)
    spec = full.with_(K=K)
    ny, nx = spec.Ny + 1, spec.Nx + 1
    units = nx * ny * spec.M * K
    res = {}

    def timed_gradient(plan, a, b, gm, reps=2):
        plan.autotune(a, b, cache=False)
        plan.set_graph(True)
        out = plan.gradient(a, b, gm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = plan.gradient(a, b, gm)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, [x.clone() for x in out]

    # batched: one plan, all combinations
    plan = rte.Plan(spec, tdt)
    a = torch.tensor(spec.mu_a, device="cuda", dtype=tdt)
    b = torch.tensor(spec.mu_s, device="cuda", dtype=tdt)
    gm = torch.zeros((plan.Nq, plan.Nd, K), device="cuda", dtype=torch.float64)
    tb, (Jb, gab, gbb, Gb) = timed_gradient(plan, a, b, gm)
    nq = plan.Nq
    res["batched"] = units * nq / tb
    log_fn("bench: MSS batched %d combinations, %d steps: %.1f ms" % (nq, K, 1000 * tb))
    plan.close()
    del plan
    torch.cuda.empty_cache()

    # plain: one plan per combination, solved one after another
    tp, ga_sum, gb_sum = 0.0, None, None
    for qc in range(nq):
        beams = [dataclasses.replace(bm, group=0) for bm in spec.beams if bm.group == qc]
        sq = spec.with_(beams=beams)
        pq = rte.Plan(sq, tdt)
        gq = torch.zeros((1, pq.Nd, K), device="cuda", dtype=torch.float64)
        t, (_, ga, gbq, _) = timed_gradient(pq, a, b, gq)
        tp += t
        ga_sum = ga if ga_sum is None else ga_sum + ga
        gb_sum = gbq if gb_sum is None else gb_sum + gbq
        pq.close()
        del pq
        torch.cuda.empty_cache()
    res["plain"] = units * nq / tp
    log_fn("bench: MSS plain %d single-combination solves: %.1f ms" % (nq, 1000 * tp))
    rel = lambda x, y: float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y))
    return {"workload": full.name, "grid": "%dx%d" % (nx, ny), "ordinates": spec.M, "combinations": nq,
            "time_steps": K, "time_steps_full": full.K, "dtype": dtype_name,
            "sample": "first %d of %d steps, every state kept (the full-length run, with checkpoints and "
                      "combination chunks, is bench.py --workload mss-full)" % (K, full.K),
            "batched_value": res["batched"], "plain_value": res["plain"],
            "unit": "cell*ordinate*steps/s", "batched_over_plain": res["batched"] / res["plain"],
            "plain_vs_batched_gradient_rel_diff": max(rel(ga_sum, gab), rel(gb_sum, gbb))}


def uneven_comparison(scale, log_fn, count=32, dtype_name="f64", keep_gradients=False):
    """The uneven batch (independent instances of different grids, ordinate
    counts and step counts; grids and steps scaled by `scale`): all instances
    in one graph launch with one branch per instance ("batched") against the
    instances one after another, each as its own recorded graph ("plain")."""
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte

    specs = W.uneven_batch(count=count, scale=scale)
    tdt = torch.float64 if dtype_name == "f64" else torch.float32
    es = 8 if dtype_name == "f64" else 4
    plans, media, gms, units = [], [], [], 0
    for sp in specs:
        ny, nx = sp.Ny + 1, sp.Nx + 1
        state = es * ny * (((nx + 3) // 4) * 4) * sp.M
        ck = 0 if (sp.K + 1) * state < 2e9 else max(8, int(math.sqrt(4 * sp.K)))
        pl = rte.Plan(sp, tdt, ckpt_every=ck)
        plans.append(pl)
        media.append((torch.tensor(sp.mu_a, device="cuda", dtype=tdt), torch.tensor(sp.mu_s, device="cuda", dtype=tdt)))
        gms.append(torch.zeros((1, pl.Nd, sp.K), device="cuda", dtype=torch.float64))
        units += nx * ny * sp.M * sp.K
    batch = rte.Batch(plans)
    t0 = time.perf_counter()
    batch.gradient(media, gms)
    torch.cuda.synchronize()
    log_fn("bench: uneven batch (%s): graph recorded and run once in %.1f s" % (dtype_name, time.perf_counter() - t0))
    t0 = time.perf_counter()
    Jb, dab, dbb, _ = batch.gradient(media, gms)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    grads = [(a.cpu().double().numpy().copy(), b.cpu().double().numpy().copy()) for a, b in zip(dab, dbb)] \
        if keep_gradients else None
    log_fn("bench: uneven batch of %d instances, one graph launch: %.1f ms" % (len(plans), 1000 * tb))
    for pl in plans:
        pl.set_graph(True)
    for pl, (a, b), g in zip(plans, media, gms):
        pl.gradient(a, b, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, (a, b), g in zip(plans, media, gms):
        pl.gradient(a, b, g)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    log_fn("bench: uneven batch, instances one after another: %.1f ms" % (1000 * tp))
    batch.close()
    for pl in plans:
        pl.close()
    torch.cuda.empty_cache()
    out = {"workload": "uneven batch of %d instances" % len(specs), "scale": scale,
            "grids": "%d..%d" % (min(s.Nx + 1 for s in specs), max(s.Nx + 1 for s in specs)),
            "ordinates": sorted(set(s.M for s in specs)), "steps": "%d..%d" % (min(s.K for s in specs), max(s.K for s in specs)),
            "dtype": dtype_name, "units": units, "batched_value": units / tb, "plain_value": units / tp,
            "unit": "cell*ordinate*steps/s", "batched_over_plain": tp / tb,
            "note": "grids and step counts scaled by %.2f from the 128..512-node, 500..3000-step batch; "
                    "instances above 2 GB of states use checkpoints (one forward replay)" % scale}
    return (out, grads) if keep_gradients else out


def full_workload(which, dtype_names, K_override, log_fn, plain=True):
    """Full-size runs of the large workloads with checkpointed replay: the
    8-combination MSS problem (513 x 513 nodes, 64 ordinates, 6000 steps) or
    the neck phantom (1025 x 1025 nodes, 64 ordinates, 4 combinations, 6000
    steps, a checkpoint every 200 steps).

    "batched": chunks of as many combinations as fit in 85 % of free device
    memory (every launch covers the whole chunk); "plain": one combination per
    chunk.  MSS: one plan whose gradient call runs every chunk (combo_chunk),
    so batched and plain gradients must agree bit for bit.  Neck: one plan and
    one gradient call per chunk (each call stays near a minute), gradients
    summed on the host, so the two sums agree to rounding only."""
    import dataclasses
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte

    full = W.config(2) if which == "mss-full" else W.neck_phantom()
    spec = full.with_(K=K_override) if K_override else full
    ckpt = 200 if which == "neck" else max(8, int(round(math.sqrt(4 * spec.K))))
    ckpt = min(ckpt, spec.K)
    split = which == "neck"
    ny, nx = spec.Ny + 1, spec.Nx + 1
    units = nx * ny * spec.M * spec.K * spec.Nq

    def sub_spec(q0, c):
        beams = [dataclasses.replace(bm, group=bm.group - q0) for bm in spec.beams if q0 <= bm.group < q0 + c]
        return spec.with_(beams=beams)

    runs = []
    for dn in dtype_names:
        tdt = torch.float64 if dn == "f64" else torch.float32
        a = torch.tensor(spec.mu_a, device="cuda", dtype=tdt)
        b = torch.tensor(spec.mu_s, device="cuda", dtype=tdt)
        free = torch.cuda.mem_get_info()[0]
        chunk = spec.Nq
        while True:
            probe = rte.Plan(sub_spec(0, chunk) if split else spec, tdt, ckpt_every=ckpt, combo_chunk=chunk)
            need = probe.workspace_bytes(True)
            probe.close()
            if need <= 0.85 * free or chunk == 1:
                break
            chunk -= 1
        n_chunks = -(-spec.Nq // chunk)
        chunk = -(-spec.Nq // n_chunks)   # same number of chunks, sizes as even as possible
        if need > 0.85 * free:
            raise RuntimeError("%s %s: one combination needs %.1f GB, %.1f GB free" % (which, dn, need / 1e9, free / 1e9))
        res = {"dtype": dn, "ckpt_every": ckpt}
        grads = {}
        for label, c in (("batched", chunk), ("plain", 1)):
            if label == "plain" and (not plain or chunk == 1):
                continue
            pieces = [(q0, min(c, spec.Nq - q0)) for q0 in range(0, spec.Nq, c)] if split else [(0, spec.Nq)]
            total, J_sum, ga_sum, gb_sum, ws_gb = 0.0, 0.0, None, None, 0.0
            for q0, cq in pieces:
                sp = sub_spec(q0, cq) if split else spec
                plan = rte.Plan(sp, tdt, ckpt_every=ckpt, combo_chunk=cq if split else c)
                sched = plan.autotune(a, b, cache=False)
                ws_gb = max(ws_gb, plan.workspace_bytes(True) / 1e9)
                log_fn("bench: %s %s %s: combinations %d..%d, combo_chunk %d, workspace %.1f GB, schedule %s" % (
                    which, dn, label, q0, q0 + cq - 1, cq if split else c, ws_gb,
                    {k: v for k, v in sched.items() if k != "cached"}))
                gm = torch.zeros((plan.Nq, plan.Nd, spec.K), device="cuda", dtype=torch.float64)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                J, ga, gb, G = plan.gradient(a, b, gm)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if not np.isfinite(float(J.item())) or not torch.isfinite(ga).all():
                    raise RuntimeError("non-finite gradient")
                total += dt
                J_sum += float(J.item())
                ga_sum = ga.clone() if ga_sum is None else ga_sum + ga
                gb_sum = gb.clone() if gb_sum is None else gb_sum + gb
                log_fn("bench: %s %s %s: gradient call %.2f s (J = %.6e)" % (which, dn, label, dt, float(J.item())))
                plan.close()
                del plan, J, ga, gb, G, gm
                torch.cuda.empty_cache()
            log_fn("bench: %s %s %s gradient: %.2f s, %.3e units/s (J = %.6e)" % (which, dn, label, total,
                                                                                  units / total, J_sum))
            res[label] = {"combo_chunk": c, "calls": len(pieces), "seconds": total, "value": units / total,
                          "J": J_sum, "workspace_GB": ws_gb, "schedule": {k: v for k, v in sched.items() if k != "cached"}}
            grads[label] = (ga_sum, gb_sum)
        if "plain" in res:
            rel = lambda x, y: float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y))
            res["batched_over_plain"] = res["batched"]["value"] / res["plain"]["value"]
            res["gradients_bitwise_equal"] = all(bool(torch.equal(x, y)) for x, y in zip(grads["batched"], grads["plain"]))
            res["gradients_max_rel_diff"] = max(rel(x, y) for x, y in zip(grads["batched"], grads["plain"]))
        runs.append(res)
        del grads
        torch.cuda.empty_cache()
    return {"workload": full.name, "grid": "%dx%d" % (nx, ny), "ordinates": spec.M, "combinations": spec.Nq,
            "detectors": len(spec.detectors), "time_steps": spec.K, "time_steps_full": full.K,
            "unit": "cell*ordinate*steps/s", "units_per_gradient": units,
            "launch": "eager (one stream); checkpoints every ckpt_every steps, segments replayed in the adjoint; "
                      + ("one gradient call per chunk of combinations" if split else "one gradient call (all chunks)"),
            "runs": runs}


def uneven_full_workload(log_fn):
    """The uneven batch at full size (32 instances, 129..513 nodes per side,
    16..64 ordinates, 500..3000 steps), FP64 and FP32, batched (one graph
    launch) against one after another, and the FP32 gradients against the
    FP64 ones."""
    import numpy as np
    import torch

    r64, g64 = uneven_comparison(1.0, log_fn, dtype_name="f64", keep_gradients=True)
    torch.cuda.empty_cache()
    r32, g32 = uneven_comparison(1.0, log_fn, dtype_name="f32", keep_gradients=True)
    rel = lambda x, y: float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))
    diffs = [max(rel(a32, a64), rel(b32, b64)) for (a32, b32), (a64, b64) in zip(g32, g64)]
    return {"workload": "uneven batch, full size", "f64": r64, "f32": r32,
            "f32_vs_f64_gradient_rel_l2": {"max": max(diffs), "median": float(np.median(diffs))}}


def inverse_workload(N, iters, log_fn, n_beams=8, n_comb=2, spacing=40.0):
    """The outer inverse loop (L-BFGS-B over a, Algorithm algfcinv) on the
    synthetic inverse phantom, TS (8 single-beam sources) against MSS (2
    staggered combinations of 4 beams): E(i) and elapsed time per iteration
    and the time each needs to reach the same error."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte
    from paper_2202_09421_amd.inverse import plan_objective, reconstruct

    runs = {}
    for mode in ("ts", "mss"):
        spec, a_bg, lo, hi = W.inverse_phantom(mode, N=N, n_beams=n_beams, n_comb=n_comb, spacing=spacing)
        state = 8 * (N + 1) * (((N + 1 + 3) // 4) * 4) * spec.M
        chunk = max(1, min(spec.Nq, int(150e9 // ((spec.K + 8) * state))))
        plan = rte.Plan(spec, torch.float64, combo_chunk=chunk)
        G = plan.forward(spec.mu_a, spec.mu_s)
        Gm = (G * torch.tensor(W.measured_noise(11, tuple(G.shape)), device="cuda")).contiguous()
        plan.autotune(torch.tensor(a_bg, device="cuda"), torch.tensor(spec.mu_s, device="cuda"), cache=False)
        fn = plan_objective(plan, spec.mu_s, Gm, graph=True)
        fn(a_bg)  # records the graph
        torch.cuda.synchronize()
        a, hist = reconstruct(fn, a_bg, lo, hi, max_iter=iters, a_true=spec.mu_a, dx=spec.dx, dy=spec.dy)
        units = (spec.Nx + 1) * (spec.Ny + 1) * spec.M * spec.K * spec.Nq
        log_fn("bench: inverse %s: %d sources, %d steps, %d iterations, %d gradients, %.1f s, E %.4f -> %.4f" % (
            mode, spec.Nq, spec.K, len(hist) - 1, hist[-1]["evals"], hist[-1]["seconds"], hist[0]["E"], hist[-1]["E"]))
        runs[mode] = {"sources": spec.Nq, "time_steps": spec.K, "units_per_gradient": units,
                      "iterations": len(hist) - 1, "gradients": hist[-1]["evals"], "seconds": hist[-1]["seconds"],
                      "E": [round(h["E"], 5) for h in hist], "t": [round(h["seconds"], 3) for h in hist]}
        plan.close()
        del plan
        torch.cuda.empty_cache()
    target = max(runs["ts"]["E"][-1], runs["mss"]["E"][-1])
    reach = {m: next(t for e, t in zip(r["E"], r["t"]) if e <= target) for m, r in runs.items()}
    return {"workload": "inverse phantom 2x2 cm, %dx%d nodes, 16 ordinates, %d beams (MSS: %d combinations, "
                        "%g ps apart), 16 detectors, 10%% noise" % (N + 1, N + 1, n_beams, n_comb, spacing),
            "optimizer": "L-BFGS-B, a in [0.1, 1] /cm, from the background", "runs": runs,
            "E_target": target, "seconds_to_E_target": reach,
            "ts_over_mss_time": reach["ts"] / max(reach["mss"], 1e-9)}


def mms_workload(log_fn):
    """The manufactured-solution convergence study of Sec. 5 (Fig. 4) on the
    device: max flux error at T = 0.5 ps on [0, 3]^2 (a = 0.35, b = 20 /cm,
    g = 0) under refinement of h, dt and the ordinates, each with the other
    two fine.  Errors against the exact flux k_Phi e^{-(x-T)^2-(y-T)^2}."""
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte
    from paper_2202_09421_amd.mms import k_phi, manufactured_inputs

    A, B = 0.35, 20.0

    def err(N, M, dt, T=0.5):
        K = int(round(T / dt))
        sp = W.small_problem(N=N, M=M, K=K, L=3.0, g=0.0, n_in=1.0, dt=dt, heterogeneous=False, a0=A,
                             b0=B).with_(n_out=1.0)
        plan = rte.Plan(sp, torch.float64)
        u0, uh, src, inflow = manufactured_inputs(sp, A, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, uK = plan.forward_ex(sp.mu_a, sp.mu_s, u0=u0, u_hist=uh, source=src, inflow=inflow)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        flux = (2.0 * math.pi / M) * uK[0].sum(dim=-1).cpu().numpy()
        x = np.arange(N + 1) * sp.dx
        X, Y = np.meshgrid(x, x)
        exact = k_phi() * np.exp(-(X - K * dt) ** 2 - (Y - K * dt) ** 2)
        plan.close()
        return float(np.abs(flux - exact).max()), sec

    def series(name, cases):
        rows = []
        for (N, M, dt) in cases:
            e, sec = err(N, M, dt)
            rows.append({"N": N, "M": M, "dt": dt, "max_flux_error": e, "seconds": round(sec, 3)})
            log_fn("bench: mms %s N=%d M=%d dt=%g: error %.3e" % (name, N, M, dt, e))
        for r0, r1 in zip(rows, rows[1:]):
            key = {"space": "N", "time": "dt", "angle": "M"}[name]
            ratio = r0[key] / r1[key] if name == "time" else r1[key] / r0[key]
            r1["observed_order"] = math.log(r0["max_flux_error"] / r1["max_flux_error"]) / math.log(ratio)
        return rows

    return {"workload": "manufactured solution (Sec. 5), [0,3]^2, T = 0.5 ps, a = 0.35, b = 20 /cm, g = 0",
            "space": series("space", [(N, 32, 0.0005) for N in (32, 64, 128, 256)]),
            "time": series("time", [(128, 32, dt) for dt in (0.04, 0.02, 0.01, 0.005)]),
            "angle": series("angle", [(128, M, 0.0005) for M in (4, 8, 12, 16)])}


def lab_flux_workload(log_fn):
    """The laboratory photon-flux simulation of Sec. 5 (Fig. 6) on the
    device: scalar-flux snapshots at 30, 100 and 170 ps of the beam entering
    [0,3]^2 at (1.5, 0); FP64 and FP32, forward throughput and a short
    profile of each snapshot (peak, centroid height)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte

    spec, steps = W.lab_flux(200, 32)
    out = {"workload": "laboratory flux simulation (Sec. 5, Fig. 6): [0,3]^2, 201x201 nodes, 32 ordinates, "
                       "a = 0.35, b = 20 /cm, g = 0.8, n = 1.4, beam at (1.5, 0), sigma_t = 30 ps",
           "dt_ps": spec.dt, "K": spec.K, "snapshot_steps": steps, "runs": {}}
    y = np.linspace(spec.ymin, spec.ymax, spec.Ny + 1)
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        plan = rte.Plan(spec, dt)
        plan.flux_snapshots(spec.mu_a, spec.mu_s, steps)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, _ = plan.flux_snapshots(spec.mu_a, spec.mu_s, steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        phi = phi[0].cpu().numpy()
        snaps = []
        for k, n in enumerate(steps):
            w = np.clip(phi[k], 0, None).sum(1)
            snaps.append({"t_ps": n * spec.dt, "peak": float(phi[k].max()), "min": float(phi[k].min()),
                          "centroid_y_cm": float((w * y).sum() / w.sum())})
        out["runs"][name] = {"seconds": round(sec, 4), "units_per_s": spec.units / sec, "snapshots": snaps}
        log_fn("bench: lab flux %s: %.3f s, %.3e units/s" % (name, sec, spec.units / sec))
        plan.close()
    return out


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline_sample(spec, target_s, cores, what):
    """Time the FP64 oracle (forward + exact adjoint gradient, all states
    kept) on the first steps of `spec` with `cores` threads (BLAS and FFT);
    returns the cpu_baseline record."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fc as ofc
    from oracle.solver import Oracle

    ofc.set_fft_workers(None if cores == 1 else cores)
    try:
        with threadpool_limits(limits=cores):
            o = Oracle(spec.with_(K=1))
            t0 = time.perf_counter()
            o.gradient(np.zeros((spec.Nq, len(spec.detectors), 1)))
            per_step = time.perf_counter() - t0
            Ks = int(max(2, min(60, target_s / max(per_step, 1e-3))))
            o = Oracle(spec.with_(K=Ks))
            t0 = time.perf_counter()
            o.gradient(np.zeros((spec.Nq, len(spec.detectors), Ks)))
            dt = time.perf_counter() - t0
    finally:
        ofc.set_fft_workers(None)
    units = (spec.Nx + 1) * (spec.Ny + 1) * spec.M * Ks * spec.Nq
    return {"value": units / dt, "unit": "cell*ordinate*steps/s", "cores": cores, "kind": "oracle",
            "sample": "first %d of %d steps of %s, forward + exact adjoint gradient with every state kept "
                      "(no replay), NumPy/SciPy FP64, %d thread(s), %.1f s" % (Ks, spec.K, what, cores, dt)}


def mss_headline(args, log_fn):
    """The batched MSS gradient (513 x 513 nodes, 64 ordinates, 8 combinations,
    6000 steps, checkpointed) sliced into --steps operation ranges, against the
    plain (one combination per launch) gradient; per-kernel launch times, the
    roofline of the dominant kernel class and of the whole path."""
    import dataclasses
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte

    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    full = W.config(2)
    spec = full.with_(K=args.workload_steps) if args.workload_steps else full
    nx, ny = spec.Nx + 1, spec.Ny + 1
    units = nx * ny * spec.M * spec.K * spec.Nq
    ckpt = min(spec.K, max(8, int(round(math.sqrt(4 * spec.K)))))
    a_true = torch.tensor(spec.mu_a, device="cuda", dtype=tdt)
    b_true = torch.tensor(spec.mu_s, device="cuda", dtype=tdt)
    a_bg = torch.full((ny, nx), 0.2, device="cuda", dtype=tdt)
    b_bg = torch.full((ny, nx), 50.0, device="cuda", dtype=tdt)

    # batched: the largest combination chunk that fits in 85 % of free HBM,
    # chunk sizes as even as possible
    free = torch.cuda.mem_get_info()[0]
    chunk = spec.Nq
    while chunk > 1 and not args.combo_chunk:
        probe = rte.Plan(spec, tdt, ckpt_every=ckpt, combo_chunk=chunk)
        need = probe.workspace_bytes(True)
        probe.close()
        if need <= 0.85 * free:
            break
        chunk -= 1
    chunk = args.combo_chunk or -(-spec.Nq // -(-spec.Nq // chunk))
    plan = rte.Plan(spec, tdt, ckpt_every=ckpt, combo_chunk=chunk)
    ws_gb = plan.workspace_bytes(True) / 1e9
    if args.schedule:
        plan.set_schedule(json.loads(args.schedule))
        sched = dict(plan.schedule(), cached=None)
    else:
        sched = plan.autotune(a_bg, b_bg, cache=args.tune_cache if args.tune_cache else False)
    sched = {k: v for k, v in sched.items() if k != "cached"}
    log_fn("bench: %s %s, %d combinations in chunks of %d, checkpoint every %d steps, workspace %.1f GB, "
           "schedule %s" % (spec.name, args.dtype, spec.Nq, chunk, ckpt, ws_gb, sched))
    G_true = plan.forward(a_true, b_true)
    noise = torch.tensor(W.measured_noise(3, tuple(G_true.shape)), device="cuda")
    Gm = (G_true * noise).contiguous()
    del G_true
    torch.cuda.synchronize()
    log_fn("bench: measurements (forward on the medium with inclusions) done")

    if args.profile_run:
        plan.gradient(a_bg, b_bg, Gm)
        torch.cuda.synchronize()
        log_fn("bench: profile run done")
        return None

    n_ops = plan.gradient_ops()
    S = args.steps
    cuts = [(i * n_ops) // S for i in range(S + 1)]
    for k in range(args.warmup):
        plan.gradient_range(a_bg, b_bg, Gm, cuts[k % S], cuts[k % S + 1])
        torch.cuda.synchronize()
        log_fn("bench: warmup slice %d done" % k)
    # per-kernel durations over the timed region: HIP events around every
    # launch of the four per-step kernel classes, on the plan's stream
    events = not args.no_kernel_events
    if events:
        rte.profile_enable(plan, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(S):
        out = plan.gradient_range(a_bg, b_bg, Gm, cuts[k], cuts[k + 1])
        if k % max(1, S // 10) == 0:
            log_fn("bench: slice %d of %d enqueued" % (k, S))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    live = rte.profile_read(plan) if events else None
    rte.profile_enable(plan, False)
    Jb, gab, gbb = (x.clone() for x in out[:3])
    log_fn("bench: batched gradient in %d slices: %.2f s (J = %.6e)" % (S, elapsed, float(Jb.item())))
    if not np.isfinite(float(Jb.item())) or not torch.isfinite(gab).all():
        raise RuntimeError("non-finite gradient")
    reps = 20
    kus_graph = plan.time_kernels(a_bg, b_bg, reps=reps)
    log_fn("bench: per-launch kernel times, graph of %d launches (us) %s" % (
        reps, {k: round(v, 1) for k, v in kus_graph.items()}))
    if live:
        kus = {k: 1000.0 * ms / n for k, (ms, n) in live.items() if n > 0}
        log_fn("bench: per-launch kernel times over the timed region (us) %s" % {k: round(v, 1) for k, v in kus.items()})
    else:
        kus = kus_graph
    plan.close()
    del plan, out
    torch.cuda.empty_cache()

    plain = None
    if not args.no_plain:
        pp = rte.Plan(spec, tdt, ckpt_every=ckpt, combo_chunk=1)
        psched = pp.autotune(a_bg, b_bg, cache=False) if not args.schedule else sched
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Jp, gap, gbp, _ = pp.gradient(a_bg, b_bg, Gm)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        rel = lambda x, y: float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y))
        plain = {"value": units / tp, "seconds": tp, "combo_chunk": 1,
                 "schedule": {k: v for k, v in psched.items() if k != "cached"},
                 "gradients_bitwise_equal": bool(torch.equal(gap, gab) and torch.equal(gbp, gbb)),
                 "J_rel_diff": abs(float(Jp.item()) - float(Jb.item())) / abs(float(Jb.item())),
                 "gradient_max_rel_diff": max(rel(gap, gab), rel(gbp, gbb))}
        log_fn("bench: plain gradient (one combination per launch): %.2f s" % tp)
        pp.close()
        del pp
        torch.cuda.empty_cache()

    # launches per gradient of each class: forward and replay steps, adjoint steps
    nch = -(-spec.Nq // chunk)
    per_grad = {"lines_fwd": 2 * spec.K * nch, "node_fwd": 2 * spec.K * nch,
                "node_adj": spec.K * nch, "lines_adj": spec.K * nch}
    upl = nx * ny * spec.M * chunk  # units per launch (a full chunk)
    word = WORD[args.dtype]
    kernels = {}
    for cls, us in kus.items():
        kernels[cls] = {"avg_us": round(us, 2), "graph_avg_us": round(kus_graph[cls], 2),
                        "launches_timed": None if not live else live[cls][1],
                        "launches_per_gradient": per_grad[cls],
                        "ms_per_gradient": round(us * per_grad[cls] / 1000.0, 1),
                        "algorithmic_GB_s": round(ALGO_WORDS[cls] * word * upl / (us * 1e-6) / 1e9, 1),
                        "compulsory_GB_s": round(KERNEL_WORDS[cls] * word * upl / (us * 1e-6) / 1e9, 1)}
    tot = sum(k["ms_per_gradient"] for k in kernels.values())
    for k in kernels.values():
        k["share"] = round(k["ms_per_gradient"] / tot, 3)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_gradient"])
    ach = kernels[dom]["algorithmic_GB_s"]
    algo_bytes = ALGO_WORDS[dom] * word * upl
    traffic = measured_traffic("mss", args.dtype, dom)
    value = units / elapsed
    path_gbs = value * PATH_WORDS_REPLAY * word / 1e9
    out = {
        "metric": "cell*ordinate*steps/s fwd+adjoint on 1 GPU, batched vs plain, at rel-L2 1e-10",
        "value": value,
        "unit": "cell*ordinate*steps/s",
        "n_gpus": 1,
        "steps": S,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / S,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": spec.name, "grid": "%dx%d" % (nx, ny), "ordinates": spec.M, "time_steps": spec.K,
                   "combinations": spec.Nq, "beams": len(spec.beams), "detectors": len(spec.detectors),
                   "path": "batched (combination chunks of %d per launch)" % chunk,
                   "states": "checkpoints every %d steps, segments replayed in the adjoint" % ckpt,
                   "step": "one of %d equal operation ranges of the gradient (%d operations); the %d timed "
                           "steps are one whole gradient" % (S, n_ops, S),
                   "launch": "eager, one stream", "workspace_GB": round(ws_gb, 1), "schedule": sched,
                   "units_per_gradient": units},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic["bytes"],
                     "kernel": dom, "algorithmic_bytes_per_unit": ALGO_WORDS[dom] * word,
                     "units_per_launch": upl, "algorithmic_bytes_per_launch": algo_bytes,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)",
                     "traffic_over_algorithmic": None if traffic is None else round(traffic["bytes"] / algo_bytes, 3),
                     "timing": ("HIP events around every launch of the kernel class on the plan's stream over "
                                "the timed steps" if live else "HIP events around a graph of 20 back-to-back "
                                "launches per kernel class on the plan's stream, after the timed steps")},
        "path_roofline": {"algorithmic_bytes_per_unit": PATH_WORDS_REPLAY * word,
                          "note": "forward 6 + replay 6 + adjoint 6 words + 1 stored state per unit",
                          "achieved_GB_s": path_gbs, "frac": path_gbs / HBM_PEAK_GBS},
        "kernels": kernels,
        "plain": plain,
        "batched_over_plain": None if plain is None else value / plain["value"],
    }
    if not args.no_cpu_baseline:
        one = spec.with_(beams=[dataclasses.replace(b, group=0) for b in spec.beams if b.group == 0])
        what = "one of the %d combinations on the full %dx%d grid, %d ordinates" % (spec.Nq, nx, ny, spec.M)
        log_fn("bench: timing the CPU oracle on a bounded sample (1 thread)")
        single = cpu_baseline_sample(one, args.cpu_seconds, 1, what)
        nc = host_cores()
        if nc > 1:
            log_fn("bench: timing the CPU oracle on a bounded sample (%d threads)" % nc)
            out["cpu_baseline"] = cpu_baseline_sample(one, args.cpu_seconds, nc, what)
            out["cpu_baseline"]["one_thread"] = {"value": single["value"], "sample": single["sample"]}
        else:
            out["cpu_baseline"] = single
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--schedule", default=None, metavar="JSON",
                    help='fixed launch schedule instead of autotuning, e.g. \'{"line_units_per_wave": 1, "line_waves_per_unit": 2}\'')
    ap.add_argument("--tune-cache", default=None, metavar="JSON",
                    help="autotuner cache file (reuse one tuned schedule across runs, e.g. profiler passes)")
    ap.add_argument("--uneven-scale", type=float, default=0.0,
                    help="grid and step scale of the uneven-batch comparison (0 skips it)")
    ap.add_argument("--mss-steps", type=int, default=0,
                    help="time steps of the batched-vs-plain MSS comparison (0 skips it)")
    ap.add_argument("--profile-run", action="store_true",
                    help="one eager gradient only (no graph, no events): the command profiled for counters")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized tensor 5 times (calibrates the HBM byte counters)")
    ap.add_argument("--inverse-n", type=int, default=128, help="with --workload inverse: intervals per side")
    ap.add_argument("--inverse-iters", type=int, default=20, help="with --workload inverse: L-BFGS-B iterations")
    ap.add_argument("--inverse-beams", type=int, default=8, help="with --workload inverse: beams on the perimeter")
    ap.add_argument("--inverse-combinations", type=int, default=2, help="with --workload inverse: MSS combinations")
    ap.add_argument("--inverse-spacing", type=float, default=40.0, help="with --workload inverse: MSS delay step (ps)")
    ap.add_argument("--workload", choices=["mss", "gradient257", "mss-full", "neck", "inverse", "mms", "lab-flux",
                                           "uneven-full"], default="mss",
                    help="mss (default): the benchmark line (batched MSS gradient, 513 x 513 x 64, 8 combinations, "
                         "6000 steps, checkpointed; a step is one slice of it); gradient257: the 257 x 257 x 32, "
                         "2000-step single-source gradient (a step is one whole gradient, graph replay); mss-full / "
                         "neck: one full-size gradient, batched and plain, FP64 and FP32 (own JSON line)")
    ap.add_argument("--workload-steps", type=int, default=0,
                    help="with --workload mss/mss-full/neck: run only the first K time steps (0 = all)")
    ap.add_argument("--no-plain", action="store_true", help="with --workload mss/mss-full/neck: skip the plain run")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="with --workload mss: no HIP events around the timed launches (kernel durations then "
                         "come from graph replays after the timed steps)")
    ap.add_argument("--combo-chunk", type=int, default=0,
                    help="with --workload mss: combinations per chunk (0 = as many as fit in 85 %% of free HBM); "
                         "profiling runs pin the chunk of the full run so kernel shapes match")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(sharding over several GPUs is a design, not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2202_09421_amd import rte

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copied %d MiB x 5" % args.copy_calibration)
        return
    if args.workload == "uneven-full":
        print(json.dumps(uneven_full_workload(log)), flush=True)
        return
    if args.workload == "mms":
        print(json.dumps(mms_workload(log)), flush=True)
        return
    if args.workload == "lab-flux":
        print(json.dumps(lab_flux_workload(log)), flush=True)
        return
    if args.workload == "inverse":
        print(json.dumps(inverse_workload(args.inverse_n, args.inverse_iters, log, args.inverse_beams,
                                          args.inverse_combinations, args.inverse_spacing)), flush=True)
        return
    if args.workload == "mss":
        out = mss_headline(args, log)
        if out is not None:
            print(json.dumps(out), flush=True)
        return
    if args.workload != "gradient257":
        dts = ["f64", "f32"] if args.workload == "mss-full" else ["f32"]
        out = full_workload(args.workload, dts, args.workload_steps, log, plain=not args.no_plain)
        print(json.dumps(out), flush=True)
        return
    spec = W.config(1)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    plan = rte.Plan(spec, tdt)
    ny, nx = spec.Ny + 1, spec.Nx + 1
    a_true = torch.tensor(spec.mu_a, device="cuda", dtype=tdt)
    b_true = torch.tensor(spec.mu_s, device="cuda", dtype=tdt)
    a_bg = torch.full((ny, nx), 0.2, device="cuda", dtype=tdt)
    b_bg = torch.full((ny, nx), 50.0, device="cuda", dtype=tdt)
    log("bench: %s, workspace %.1f GB" % (spec.name, plan.workspace_bytes(True) / 1e9))
    if args.schedule:
        plan.set_schedule(json.loads(args.schedule))
        sched = dict(plan.schedule(), cached=None)
    else:
        sched = plan.autotune(a_bg, b_bg, cache=args.tune_cache if args.tune_cache else False)
    log("bench: autotuned schedule %s" % sched)
    G_true = plan.forward(a_true, b_true)
    noise = torch.tensor(W.measured_noise(1, tuple(G_true.shape)), device="cuda")
    Gm = (G_true * noise).contiguous()
    torch.cuda.synchronize()

    if args.profile_run:
        plan.gradient(a_bg, b_bg, Gm)
        torch.cuda.synchronize()
        log("bench: profile run done")
        return

    # (1) one eager gradient (kernels launched one by one)
    t0 = time.perf_counter()
    plan.gradient(a_bg, b_bg, Gm)
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t0
    log("bench: eager gradient %.1f ms" % (1000 * eager_s))

    # (2) the measured steps: the whole gradient recorded once as a HIP graph
    plan.set_graph(True)
    for k in range(args.warmup):
        plan.gradient(a_bg, b_bg, Gm)
        torch.cuda.synchronize()
        log("bench: warmup %d done" % k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        J, ga, gb, G = plan.gradient(a_bg, b_bg, Gm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("bench: timed %d gradients in %.3f s (J = %.6e)" % (args.steps, elapsed, float(J.item())))
    if not np.isfinite(float(J.item())) or not torch.isfinite(ga).all():
        raise RuntimeError("non-finite gradient")

    # the paper's own gradient (continuous adjoint, always eager) on the same
    # workload, against the exact discrete one just computed
    ga_ref, gb_ref = ga.clone(), gb.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Jc, gac, gbc, _ = plan.gradient_continuous(a_bg, b_bg, Gm)
    torch.cuda.synchronize()
    cont_s = time.perf_counter() - t0
    log("bench: continuous-adjoint gradient (eager) %.1f ms" % (1000 * cont_s))
    cont = {"ms": 1000 * cont_s, "value": nx * ny * spec.M * spec.K * spec.Nq / cont_s,
            "unit": "cell*ordinate*steps/s", "eager_discrete_ms": 1000 * eager_s,
            "J_equal": bool(torch.equal(Jc, J)),
            "dir_derivative_rel_diff": {
                "da=1": abs(float(gac.sum() - ga_ref.sum())) / abs(float(ga_ref.sum())),
                "db=1": abs(float(gbc.sum() - gb_ref.sum())) / abs(float(gb_ref.sum()))},
            "note": "eq. (AdjointProblem) solved by the forward kernels in reversed time and ordinates, "
                    "eq. (FDwin22) in the node pass; differs from the exact discrete gradient by "
                    "discretisation error"}
    del gac, gbc, ga_ref, gb_ref

    # (3) per-kernel durations (roofline figures), right after the timed
    #     steps on the same stream: for each kernel class, 20 back-to-back
    #     launches on the benchmark's shapes recorded as one graph and timed
    #     between HIP events (rte_plan_time_kernels)
    reps = 20
    kus = plan.time_kernels(a_bg, b_bg, reps=reps)
    log("bench: per-launch kernel times (us) %s" % {k: round(v, 2) for k, v in kus.items()})
    prof = {k: (v * reps / 1000.0, reps) for k, v in kus.items()}

    units_per_grad = nx * ny * spec.M * spec.K * spec.Nq
    ms_per_step = 1000.0 * elapsed / args.steps
    value = units_per_grad * args.steps / elapsed

    word = WORD[args.dtype]
    units_per_launch = nx * ny * spec.M * spec.Nq
    kernels = {}
    for cls, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_us = 1000.0 * ms / cnt
        gbs = KERNEL_WORDS[cls] * word * units_per_launch / (avg_us * 1e-6) / 1e9
        kernels[cls] = {"avg_us": round(avg_us, 2), "launches": cnt, "GB_s": round(gbs, 1),
                        "share": round(ms / max(1e-9, sum(v[0] for v in prof.values())), 3)}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    ach = kernels[dom]["GB_s"]
    path_gbs = value * PATH_WORDS_STORE_ALL * word / 1e9
    bytes_per_launch = KERNEL_WORDS[dom] * word * units_per_launch
    traffic = measured_traffic("gradient257", args.dtype, dom)
    out = {
        "metric": "cell*ordinate*steps/s fwd+adjoint on 1 GPU, batched vs plain, at rel-L2 1e-10",
        "value": value,
        "unit": "cell*ordinate*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": spec.name, "grid": "%dx%d" % (nx, ny), "ordinates": spec.M, "time_steps": spec.K,
                   "sources": spec.Nq, "detectors": len(spec.detectors), "states": "all kept (no replay)",
                   "path": "plain (one source: batched == plain)", "launch": "one HIP graph per gradient",
                   "schedule": {k: v for k, v in sched.items() if k != "cached"},
                   "eager_ms_per_step": round(1000 * eager_s, 2)},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic["bytes"],
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
                     "traffic_over_algorithmic": None if traffic is None else round(traffic["bytes"] / bytes_per_launch, 3),
                     "kernel": dom,
                     "bytes_per_launch": bytes_per_launch,
                     "timing": "HIP events around a graph of 20 back-to-back launches per kernel class, after the timed steps"},
        "path_roofline": {"algorithmic_bytes_per_unit": PATH_WORDS_STORE_ALL * word, "achieved_GB_s": path_gbs,
                          "frac": path_gbs / HBM_PEAK_GBS},
        "kernels": kernels,
        "continuous_adjoint": cont,
    }
    if args.mss_steps > 0 or args.uneven_scale > 0:
        plan.close()
        del plan
        torch.cuda.empty_cache()
    if args.mss_steps > 0:
        out["mss_batched_vs_plain"] = mss_comparison(args.mss_steps, args.dtype, log)
    if args.uneven_scale > 0:
        out["uneven_batched_vs_plain"] = uneven_comparison(args.uneven_scale, log)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
