"""Python binding of librte.so (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; this module turns a
problem description into the C structs, allocates outputs and the workspace
with torch on the current CUDA (HIP) device, and passes raw pointers plus the
current stream.  It never computes any part of the method itself and raises if
the library is missing: there is no CPU fallback.

Problem descriptions are duck-typed: any object with the fields of the C
``rte_problem`` (xmin, xmax, ymin, ymax, Nx, Ny, M, K, dt, c, g, hg_exponent,
n_in, n_out, fc_d, fc_C, filt_alpha, filt_beta), a list ``beams`` (x, y,
theta, sigma_x, sigma_theta, tau, sigma_t, t0, group) and a list
``detectors`` (x, y, sigma_d).
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librte.so")

RTE_OK, RTE_EINVAL, RTE_ENOMEM, RTE_EDEVICE, RTE_EUNSTABLE, RTE_EUNSUPPORTED, RTE_ESTATE = 0, -1, -2, -3, -4, -5, -6
RTE_F64, RTE_F32 = 0, 1


class RteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rte error %d: %s" % (code, msg))
        self.code = code


class rte_problem(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("Nx", ctypes.c_int64), ("Ny", ctypes.c_int64), ("M", ctypes.c_int64), ("K", ctypes.c_int64),
                ("xmin", ctypes.c_double), ("xmax", ctypes.c_double), ("ymin", ctypes.c_double),
                ("ymax", ctypes.c_double), ("c", ctypes.c_double), ("dt", ctypes.c_double),
                ("g", ctypes.c_double), ("hg_exponent", ctypes.c_double), ("n_in", ctypes.c_double),
                ("n_out", ctypes.c_double), ("fc_d", ctypes.c_int64), ("fc_C", ctypes.c_int64),
                ("filt_alpha", ctypes.c_double), ("filt_beta", ctypes.c_double),
                ("fc_Q", ctypes.POINTER(ctypes.c_double)), ("fc_A", ctypes.POINTER(ctypes.c_double)),
                ("ckpt_every", ctypes.c_int64), ("combo_chunk", ctypes.c_int64)]


class rte_beam(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("x", "y", "theta", "sigma_x", "sigma_theta", "tau", "sigma_t", "t0")] + \
               [("group", ctypes.c_int32), ("profile", ctypes.c_int32)]


RTE_PROFILE = {"gauss": 0, "window": 1}


class rte_detector(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("sigma_d", ctypes.c_double)]


class rte_schedule(ctypes.Structure):
    _fields_ = [("line_units_per_wave", ctypes.c_int32), ("line_generic", ctypes.c_int32),
                ("node_tiles_per_block", ctypes.c_int32), ("line_waves_per_unit", ctypes.c_int32),
                ("line_global_tables", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"line_units_per_wave": self.line_units_per_wave, "line_generic": self.line_generic,
                "node_tiles_per_block": self.node_tiles_per_block, "line_waves_per_unit": self.line_waves_per_unit,
                "line_global_tables": self.line_global_tables}


_lib = None


class rte_separable(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("X", ctypes.c_void_p),
                ("Y", ctypes.c_void_p), ("Th", ctypes.c_void_p)]


class rte_forward_extra(ctypes.Structure):
    _fields_ = [("u0", ctypes.c_void_p), ("u_hist", ctypes.c_void_p), ("source", rte_separable),
                ("inflow", rte_separable), ("n_snap", ctypes.c_int32), ("reserved1", ctypes.c_int32),
                ("snap_steps", ctypes.POINTER(ctypes.c_int32)), ("snap_flux", ctypes.c_void_p)]


def lib():
    """Load librte.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librte.so not found at %s: run paper_2202_09421_amd.build.build() first" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        L.rte_plan_create.argtypes = [ctypes.POINTER(rte_problem), ctypes.POINTER(rte_beam), i64,
                                      ctypes.POINTER(rte_detector), i64, ctypes.POINTER(vp)]
        L.rte_plan_destroy.argtypes = [vp]
        L.rte_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.rte_workspace_bytes.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64)]
        L.rte_forward.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp, i64, vp]
        L.rte_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, vp]
        L.rte_gradient.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp]
        L.rte_gradient_continuous.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp]
        L.rte_gradient_ops.argtypes = [vp, ctypes.POINTER(i64)]
        L.rte_gradient_range.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, i64, vp]
        L.rte_forward_ex.argtypes = [vp, vp, vp, ctypes.POINTER(rte_forward_extra), vp, vp, vp, i64, vp]
        L.rte_plan_set_graph.argtypes = [vp, ctypes.c_int]
        L.rte_plan_set_guard.argtypes = [vp, ctypes.c_int]
        L.rte_batch_create.argtypes = [ctypes.POINTER(vp), i64, ctypes.POINTER(vp)]
        L.rte_batch_destroy.argtypes = [vp]
        pp = ctypes.POINTER(vp)
        L.rte_batch_gradient.argtypes = [vp, pp, pp, pp, pp, pp, pp, pp, pp, ctypes.POINTER(i64), vp]
        L.rte_profile_enable.argtypes = [vp, ctypes.c_int]
        L.rte_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        sp = ctypes.POINTER(rte_schedule)
        L.rte_plan_get_schedule.argtypes = [vp, sp]
        L.rte_plan_set_schedule.argtypes = [vp, sp]
        L.rte_plan_autotune.argtypes = [vp, vp, vp, vp, i64, vp, sp]
        L.rte_plan_time_kernels.argtypes = [vp, vp, vp, vp, i64, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.rte_last_error.restype = ctypes.c_char_p
        for f in ("rte_plan_create", "rte_plan_destroy", "rte_plan_info", "rte_workspace_bytes", "rte_forward",
                  "rte_adjoint", "rte_gradient", "rte_profile_enable", "rte_profile_read", "rte_plan_set_graph",
                  "rte_batch_create", "rte_batch_destroy", "rte_batch_gradient", "rte_plan_get_schedule",
                  "rte_plan_set_schedule", "rte_plan_autotune", "rte_plan_time_kernels", "rte_gradient_continuous",
                  "rte_forward_ex", "rte_plan_set_guard", "rte_gradient_ops", "rte_gradient_range"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != RTE_OK:
        raise RteError(rc, lib().rte_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_problem(spec, dtype=RTE_F64, ckpt_every=0, combo_chunk=0, fc_QA=None):
    """Build the C structs for a problem description (see module docstring).
    fc_QA: optional (Q [d, d], A [C, d]) FC table; None uses the library's
    built-in table (d = 5, C = 25)."""
    p = rte_problem()
    p.dtype = dtype
    p.Nx, p.Ny, p.M, p.K = spec.Nx, spec.Ny, spec.M, spec.K
    p.xmin, p.xmax, p.ymin, p.ymax = spec.xmin, spec.xmax, spec.ymin, spec.ymax
    p.c, p.dt, p.g, p.hg_exponent = spec.c, spec.dt, spec.g, spec.hg_exponent
    p.n_in, p.n_out = spec.n_in, spec.n_out
    p.fc_d, p.fc_C = spec.fc_d, spec.fc_C
    p.filt_alpha, p.filt_beta = spec.filt_alpha, spec.filt_beta
    keep = ()
    if fc_QA is not None:
        Qc = np.ascontiguousarray(fc_QA[0], dtype=np.float64)
        Ac = np.ascontiguousarray(fc_QA[1], dtype=np.float64)
        p.fc_Q = Qc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.fc_A = Ac.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep = (Qc, Ac)
    p.ckpt_every = ckpt_every
    p.combo_chunk = combo_chunk
    beams = (rte_beam * max(1, len(spec.beams)))()
    for k, b in enumerate(spec.beams):
        beams[k] = rte_beam(b.x, b.y, b.theta, b.sigma_x, b.sigma_theta, b.tau, b.sigma_t, b.t0, b.group,
                            RTE_PROFILE[getattr(b, "profile", "gauss")])
    dets = (rte_detector * max(1, len(spec.detectors)))()
    for k, dd in enumerate(spec.detectors):
        dets[k] = rte_detector(dd.x, dd.y, dd.sigma_d)
    return p, beams, len(spec.beams), dets, len(spec.detectors), keep


class Plan:
    """A library plan for one problem description (all Nq sources)."""

    def __init__(self, spec, dtype=torch.float64, ckpt_every=0, device=None, combo_chunk=0, fc_QA=None):
        self.spec = spec
        self.dtype = dtype
        self.device = torch.device("cuda") if device is None else torch.device(device)
        code = RTE_F64 if dtype == torch.float64 else RTE_F32
        prob, beams, nb, dets, nd, self._keep = make_problem(spec, code, ckpt_every, combo_chunk, fc_QA)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().rte_plan_create(ctypes.byref(prob), beams, nb, dets, nd, ctypes.byref(h)))
        self._h = h
        Nq, Nd, Npx, Npy = (ctypes.c_int64() for _ in range(4))
        _check(lib().rte_plan_info(h, ctypes.byref(Nq), ctypes.byref(Nd), ctypes.byref(Npx), ctypes.byref(Npy)))
        self.Nq, self.Nd, self.Np_x, self.Np_y = Nq.value, Nd.value, Npx.value, Npy.value
        self._ws = None
        self._graph = False
        self._gout = None
        # bumped by every call that rewrites the workspace; RTEFunction
        # checks it to know whether its saved forward is still there
        self.generation = 0

    def close(self):
        """Destroy the library plan and drop the workspace and output buffers
        (their memory returns to torch's allocator)."""
        if getattr(self, "_h", None):
            lib().rte_plan_destroy(self._h)
            self._h = None
        self._ws = None
        self._gout = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, with_adjoint=True):
        b = ctypes.c_int64()
        _check(lib().rte_workspace_bytes(self._h, 1 if with_adjoint else 0, ctypes.byref(b)))
        return b.value

    def workspace(self, with_adjoint=True):
        need = self.workspace_bytes(with_adjoint)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def _medium(self, mu_a, mu_s):
        ny, nx = self.spec.Ny + 1, self.spec.Nx + 1
        a = torch.as_tensor(mu_a, dtype=self.dtype, device=self.device).contiguous()
        b = torch.as_tensor(mu_s, dtype=self.dtype, device=self.device).contiguous()
        if a.shape != (ny, nx) or b.shape != (ny, nx):
            raise ValueError("mu_a and mu_s must have shape (Ny+1, Nx+1)")
        return a, b

    def forward(self, mu_a, mu_s, save_states=False, want_u_final=False):
        a, b = self._medium(mu_a, mu_s)
        G = torch.empty((self.Nq, self.Nd, self.spec.K), dtype=torch.float64, device=self.device)
        uK = None
        if want_u_final:
            uK = torch.empty((self.Nq, self.spec.Ny + 1, self.spec.Nx + 1, self.spec.M), dtype=self.dtype,
                             device=self.device)
        ws = self.workspace(save_states)
        self.generation += 1
        _check(lib().rte_forward(self._h, _ptr(a), _ptr(b), _ptr(G), _ptr(uK), 1 if save_states else 0,
                                 _ptr(ws), ws.numel(), _stream()))
        self._medium_saved = (a, b)
        return (G, uK) if want_u_final else G

    def adjoint(self, G_bar, mu_a=None, mu_s=None):
        if mu_a is None:
            a, b = self._medium_saved
        else:
            a, b = self._medium(mu_a, mu_s)
        gbar = torch.as_tensor(G_bar, dtype=torch.float64, device=self.device).contiguous()
        ny, nx = self.spec.Ny + 1, self.spec.Nx + 1
        da = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        db = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        ws = self.workspace(True)
        _check(lib().rte_adjoint(self._h, _ptr(a), _ptr(b), _ptr(gbar), _ptr(da), _ptr(db), _ptr(ws), ws.numel(),
                                 _stream()))
        return da, db

    def schedule(self):
        """Current launch schedule (dict)."""
        sc = rte_schedule()
        _check(lib().rte_plan_get_schedule(self._h, ctypes.byref(sc)))
        return sc.as_dict()

    def set_schedule(self, sched):
        sc = rte_schedule(int(sched.get("line_units_per_wave", 0)), int(sched.get("line_generic", 0)),
                          int(sched.get("node_tiles_per_block", 0)), int(sched.get("line_waves_per_unit", 0)),
                          int(sched.get("line_global_tables", 0)), 0)
        _check(lib().rte_plan_set_schedule(self._h, ctypes.byref(sc)))

    def tune_key(self):
        sp = self.spec
        dev = torch.cuda.get_device_name(self.device) if torch.cuda.is_available() else "none"
        return "%s|%s|nx%d|ny%d|M%d|Nq%d|Np%d,%d" % (dev, "f64" if self.dtype == torch.float64 else "f32",
                                                     sp.Nx + 1, sp.Ny + 1, sp.M, self.Nq, self.Np_x, self.Np_y)

    def autotune(self, mu_a, mu_s, cache=None):
        """Pick the fastest launch schedule for this plan's shapes with the
        library's autotuner (rte_plan_autotune) and apply it.  `cache`: a JSON
        file of earlier choices keyed by device and shapes (default
        $RTE_TUNE_CACHE or ~/.cache/rte_fcdom/schedules.json; False disables);
        a hit applies the stored schedule without timing."""
        path = None
        if cache is not False:
            path = cache or os.environ.get("RTE_TUNE_CACHE") or os.path.join(
                os.path.expanduser("~"), ".cache", "rte_fcdom", "schedules.json")
        key = self.tune_key()
        table = {}
        if path and os.path.exists(path):
            try:
                with open(path) as fh:
                    table = json.load(fh)
            except (OSError, ValueError):
                table = {}
        if key in table:
            self.set_schedule(table[key])
            return dict(table[key], cached=True)
        a, b = self._medium(mu_a, mu_s)
        ws = self.workspace(True)
        sc = rte_schedule()
        self.generation += 1
        _check(lib().rte_plan_autotune(self._h, _ptr(a), _ptr(b), _ptr(ws), ws.numel(), _stream(), ctypes.byref(sc)))
        chosen = sc.as_dict()
        if path:
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                table[key] = chosen
                tmp = path + ".tmp%d" % os.getpid()
                with open(tmp, "w") as fh:
                    json.dump(table, fh, indent=1, sort_keys=True)
                os.replace(tmp, path)
            except OSError:
                pass
        return dict(chosen, cached=False)

    def time_kernels(self, mu_a, mu_s, reps=20):
        """Microseconds per launch of each kernel class (KERNEL_CLASSES) with
        the current schedule, from graph replays of back-to-back launches
        (rte_plan_time_kernels).  Overwrites the workspace."""
        a, b = self._medium(mu_a, mu_s)
        ws = self.workspace(True)
        us = (ctypes.c_double * len(KERNEL_CLASSES))()
        self.generation += 1
        _check(lib().rte_plan_time_kernels(self._h, _ptr(a), _ptr(b), _ptr(ws), ws.numel(), _stream(), int(reps), us))
        return {k: us[i] for i, k in enumerate(KERNEL_CLASSES)}

    def set_guard(self, on=True):
        """Non-finite guard (rte_plan_set_guard): every call then scans its
        FP64 outputs after the solve, waits for the stream and raises RteError
        with code RTE_EUNSTABLE if any value is NaN or infinite."""
        _check(lib().rte_plan_set_guard(self._h, 1 if on else 0))

    def set_graph(self, on=True):
        """Graph mode: rte_gradient is recorded once per argument set and
        replayed.  Outputs then live in buffers owned by the plan (reused by
        every call: copy them to keep a result across calls), and inputs must
        be the same tensors from call to call to avoid re-recording."""
        _check(lib().rte_plan_set_graph(self._h, 1 if on else 0))
        self._graph = bool(on)

    def _outputs(self):
        ny, nx = self.spec.Ny + 1, self.spec.Nx + 1
        mk = lambda *sh: torch.empty(sh, dtype=torch.float64, device=self.device)
        if not self._graph:
            return mk(1), mk(ny, nx), mk(ny, nx), mk(self.Nq, self.Nd, self.spec.K)
        if self._gout is None:
            self._gout = (mk(1), mk(ny, nx), mk(ny, nx), mk(self.Nq, self.Nd, self.spec.K))
        return self._gout

    def gradient(self, mu_a, mu_s, G_meas):
        a, b = self._medium(mu_a, mu_s)
        gm = torch.as_tensor(G_meas, dtype=torch.float64, device=self.device).contiguous()
        J, da, db, G = self._outputs()
        ws = self.workspace(True)
        self.generation += 1
        _check(lib().rte_gradient(self._h, _ptr(a), _ptr(b), _ptr(gm), _ptr(J), _ptr(da), _ptr(db), _ptr(G),
                                  _ptr(ws), ws.numel(), _stream()))
        return J, da, db, G

    def gradient_ops(self):
        """Number of operations of one gradient (rte_gradient_ops)."""
        n = ctypes.c_int64()
        _check(lib().rte_gradient_ops(self._h, ctypes.byref(n)))
        return n.value

    def gradient_range(self, mu_a, mu_s, G_meas, first, last):
        """Enqueue operations [first, last) of one gradient (rte_gradient_range).
        Ranges of one gradient go in order from 0 with the same tensors; the
        outputs (J, dmu_a, dmu_s, G), owned by the plan and reused by every
        staged gradient, are complete after the range holding the last op."""
        a, b = self._medium(mu_a, mu_s)
        gm = torch.as_tensor(G_meas, dtype=torch.float64, device=self.device).contiguous()
        if first == 0 or getattr(self, "_rng", None) is None:
            ny, nx = self.spec.Ny + 1, self.spec.Nx + 1
            mk = lambda *sh: torch.empty(sh, dtype=torch.float64, device=self.device)
            if getattr(self, "_rng_out", None) is None:
                self._rng_out = (mk(1), mk(ny, nx), mk(ny, nx), mk(self.Nq, self.Nd, self.spec.K))
            self._rng = (a, b, gm)   # the inputs stay alive (and equal) for the whole sequence
        a, b, gm = self._rng
        J, da, db, G = self._rng_out
        ws = self.workspace(True)
        self.generation += 1
        _check(lib().rte_gradient_range(self._h, _ptr(a), _ptr(b), _ptr(gm), _ptr(J), _ptr(da), _ptr(db), _ptr(G),
                                        _ptr(ws), ws.numel(), int(first), int(last), _stream()))
        return J, da, db, G


    def forward_ex(self, mu_a, mu_s, u0=None, u_hist=None, source=None, inflow=None, want_u_final=True):
        """rte_forward_ex: forward solve with an initial state u0 [Nq, ny, nx, M],
        start-up states u_hist [3, Nq, ny, nx, M] (t_{-1}, t_{-2}, t_{-3}), a
        volumetric source and inflow data, each a separable field (X [R, K+4, nx],
        Y [R, K+4, ny], Th [R, M]) on the time levels -3..K, or None."""
        G, uK, _ = self._forward_ex(mu_a, mu_s, u0, u_hist, source, inflow, want_u_final, None)
        return (G, uK) if want_u_final else G

    def flux_snapshots(self, mu_a, mu_s, steps, u0=None, u_hist=None, source=None, inflow=None):
        """Scalar flux phi(x, t_n) = dtheta sum_m u_m (eq. photondensity) of the
        forward states u^n at the time levels `steps` (each in [0, K]), as in
        Fig. 6: returns (phi [Nq, len(steps), ny, nx] FP64, G).  Other
        arguments as in forward_ex."""
        G, _, phi = self._forward_ex(mu_a, mu_s, u0, u_hist, source, inflow, False, steps)
        return phi, G

    def _forward_ex(self, mu_a, mu_s, u0, u_hist, source, inflow, want_u_final, snap_steps):
        a, b = self._medium(mu_a, mu_s)
        keep = []

        def dev(x, dtype):
            if x is None:
                return None
            t = torch.as_tensor(x, dtype=dtype, device=self.device).contiguous()
            keep.append(t)
            return t

        def sep(f):
            out = rte_separable()
            if f is None:
                return out
            X, Y, Th = (dev(v, torch.float64) for v in f)
            K4, nx, ny = self.spec.K + 4, self.spec.Nx + 1, self.spec.Ny + 1
            R = X.shape[0]
            if X.shape != (R, K4, nx) or Y.shape != (R, K4, ny) or Th.shape != (R, self.spec.M):
                raise ValueError("separable field shapes must be [R, K+4, nx], [R, K+4, ny], [R, M]")
            out.rank, out.X, out.Y, out.Th = R, _ptr(X), _ptr(Y), _ptr(Th)
            return out

        ex = rte_forward_extra()
        ex.u0 = _ptr(dev(u0, self.dtype)) if u0 is not None else None
        ex.u_hist = _ptr(dev(u_hist, self.dtype)) if u_hist is not None else None
        ex.source = sep(source)
        ex.inflow = sep(inflow)
        phi = None
        if snap_steps is not None:
            steps = np.ascontiguousarray(np.asarray(snap_steps, dtype=np.int32).reshape(-1))
            phi = torch.empty((self.Nq, steps.size, self.spec.Ny + 1, self.spec.Nx + 1), dtype=torch.float64,
                              device=self.device)
            ex.n_snap = steps.size
            ex.snap_steps = steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            ex.snap_flux = _ptr(phi)
        G = torch.empty((self.Nq, self.Nd, self.spec.K), dtype=torch.float64, device=self.device)
        uK = None
        if want_u_final:
            uK = torch.empty((self.Nq, self.spec.Ny + 1, self.spec.Nx + 1, self.spec.M), dtype=self.dtype,
                             device=self.device)
        ws = self.workspace(False)
        self.generation += 1
        _check(lib().rte_forward_ex(self._h, _ptr(a), _ptr(b), ctypes.byref(ex), _ptr(G), _ptr(uK), _ptr(ws),
                                    ws.numel(), _stream()))
        # the tables in `keep` may be released now: later allocations reuse
        # their memory in stream order, after these kernels
        return G, uK, phi

    def gradient_continuous(self, mu_a, mu_s, G_meas):
        """J, dJ/dmu_a, dJ/dmu_s, G by the paper's continuous adjoint
        (rte_gradient_continuous): equal to `gradient` in J and G, and in the
        gradient maps to discretisation error.  Always eager."""
        a, b = self._medium(mu_a, mu_s)
        gm = torch.as_tensor(G_meas, dtype=torch.float64, device=self.device).contiguous()
        ny, nx = self.spec.Ny + 1, self.spec.Nx + 1
        mk = lambda *sh: torch.empty(sh, dtype=torch.float64, device=self.device)
        J, da, db, G = mk(1), mk(ny, nx), mk(ny, nx), mk(self.Nq, self.Nd, self.spec.K)
        ws = self.workspace(True)
        self.generation += 1
        _check(lib().rte_gradient_continuous(self._h, _ptr(a), _ptr(b), _ptr(gm), _ptr(J), _ptr(da), _ptr(db),
                                             _ptr(G), _ptr(ws), ws.numel(), _stream()))
        return J, da, db, G


class Batch:
    """Uneven batch: rte_gradient of several plans in one graph launch.
    Inputs must stay the same tensors between calls (the graph is replayed
    while every pointer is unchanged); outputs are owned by the batch."""

    def __init__(self, plans):
        self.plans = list(plans)
        hs = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().rte_batch_create(hs, len(self.plans), ctypes.byref(h)))
        self._h = h
        self._out = None

    def close(self):
        if getattr(self, "_h", None):
            lib().rte_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gradient(self, media, G_meas):
        """media: list of (mu_a, mu_s); G_meas: list.  Returns lists J, dmu_a, dmu_s, G."""
        n = len(self.plans)
        ins = [p._medium(a, b) for p, (a, b) in zip(self.plans, media)]
        gms = [torch.as_tensor(g, dtype=torch.float64, device=p.device).contiguous() for p, g in zip(self.plans, G_meas)]
        if self._out is None:
            self._out = [p._outputs() if p._graph else
                         (lambda P: (torch.empty(1, dtype=torch.float64, device=P.device),
                                     torch.empty((P.spec.Ny + 1, P.spec.Nx + 1), dtype=torch.float64, device=P.device),
                                     torch.empty((P.spec.Ny + 1, P.spec.Nx + 1), dtype=torch.float64, device=P.device),
                                     torch.empty((P.Nq, P.Nd, P.spec.K), dtype=torch.float64, device=P.device)))(p)
                         for p in self.plans]
        wss = [p.workspace(True) for p in self.plans]
        self._keep = (ins, gms)
        arr = lambda xs: (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        J = [o[0] for o in self._out]
        da = [o[1] for o in self._out]
        db = [o[2] for o in self._out]
        G = [o[3] for o in self._out]
        wb = (ctypes.c_int64 * n)(*[w.numel() for w in wss])
        for p in self.plans:
            p.generation += 1
        _check(lib().rte_batch_gradient(self._h, arr([x[0] for x in ins]), arr([x[1] for x in ins]), arr(gms),
                                        arr(J), arr(da), arr(db), arr(G), arr(wss), wb, _stream()))
        return J, da, db, G


KERNEL_CLASSES = ("lines_fwd", "node_fwd", "node_adj", "lines_adj")


def profile_enable(plan, on=True):
    _check(lib().rte_profile_enable(plan._h, 1 if on else 0))


def profile_read(plan):
    """{class: (total_ms, launches)} since the last read (waits for the GPU)."""
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().rte_profile_read(plan._h, ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}


class RTEFunction(torch.autograd.Function):
    """G = F(mu_a, mu_s): detector traces [Nq, Nd, K] of the forward solve.
    backward runs the library's exact discrete adjoint (checkpointed replay
    when the plan was made with ckpt_every > 0).  If another call rewrote the
    plan's workspace after this forward (a second application of the
    Function, a gradient, a line-search trial), backward first re-runs the
    forward with the saved medium so that the adjoint pairs with its own
    states."""

    @staticmethod
    def forward(ctx, mu_a, mu_s, plan):
        ctx.plan = plan
        ctx.save_for_backward(mu_a, mu_s)
        G = plan.forward(mu_a.detach(), mu_s.detach(), save_states=True)
        ctx.generation = plan.generation
        return G

    @staticmethod
    def backward(ctx, grad_G):
        mu_a, mu_s = ctx.saved_tensors
        plan = ctx.plan
        if plan.generation != ctx.generation:
            plan.forward(mu_a.detach(), mu_s.detach(), save_states=True)
        da, db = plan.adjoint(grad_G.contiguous(), mu_a.detach(), mu_s.detach())
        return da.to(mu_a.dtype), db.to(mu_s.dtype), None


def detector_traces(mu_a, mu_s, plan):
    return RTEFunction.apply(mu_a, mu_s, plan)
