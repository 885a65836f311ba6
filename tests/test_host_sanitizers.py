"""CPU: the library's host code (problem validation, ordinate / HG / Fresnel /
beam / detector / FC table construction, argument checks of the entry
points) under AddressSanitizer and UndefinedBehaviorSanitizer.  Without a
GPU, a valid plan is built up to the device upload (which then fails with
RTE_EDEVICE), so every host table of the configurations below is built and
checked."""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = textwrap.dedent("""
    import ctypes, sys
    sys.path.insert(0, %(root)r)
    import workloads as W
    from paper_2202_09421_amd import rte
    rte.LIB_PATH = %(lib)r
    L = rte.lib()
    specs = [W.small_problem(N=12, M=8, K=4), W.small_problem(N=9, M=4, K=3, Ny=9),
             W.small_problem(N=20, M=48, K=5, Ny=13, n_in=1.33), W.small_problem(N=12, M=80, K=2, n_in=1.0),
             W.config(0), W.config(1), W.lab_flux(24, 8)[0], W.inverse_phantom()[0],
             W.small_problem(N=1024, M=4, K=2, Ny=9), W.small_problem(N=9, M=8, K=2, Ny=700)]
    for s in specs:
        prob, beams, nb, dets, nd, keep = rte.make_problem(s)
        h = ctypes.c_void_p()
        rc = L.rte_plan_create(ctypes.byref(prob), beams, nb, dets, nd, ctypes.byref(h))
        assert rc in (rte.RTE_OK, rte.RTE_EDEVICE), (s.name, rc, L.rte_last_error())
    # invalid descriptions and NULL arguments
    s = W.small_problem(N=12, M=8, K=4)
    for field, value in (("M", 6), ("Nx", 5), ("K", 0), ("g", 1.0), ("dt", -1.0), ("dt", 50.0), ("dtype", 7)):
        prob, beams, nb, dets, nd, keep = rte.make_problem(s)
        setattr(prob, field, value)
        h = ctypes.c_void_p()
        assert L.rte_plan_create(ctypes.byref(prob), beams, nb, dets, nd, ctypes.byref(h)) == rte.RTE_EINVAL
    prob, beams, nb, dets, nd, keep = rte.make_problem(s)
    beams[0].x, beams[0].y = 0.5, 0.5
    assert L.rte_plan_create(ctypes.byref(prob), beams, nb, dets, nd, ctypes.byref(ctypes.c_void_p())) == rte.RTE_EINVAL
    assert L.rte_plan_create(None, None, 0, None, 0, None) == rte.RTE_EINVAL
    assert L.rte_forward(None, None, None, None, None, 0, None, 0, None) == rte.RTE_EINVAL
    assert L.rte_forward_ex(None, None, None, None, None, None, None, 0, None) == rte.RTE_EINVAL
    assert L.rte_plan_set_guard(None, 1) == rte.RTE_EINVAL
    print("host checks done", flush=True)
""")


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2202_09421_amd import build as B
    rt = _asan_runtime()
    if rt is None or not os.path.exists(B._hipcc()):
        pytest.skip("no hipcc or ASan runtime")
    if not all(os.path.exists(os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o")) for s in B.SOURCES):
        B.build()
    lib = B.build_host_sanitized(str(tmp_path))
    script = tmp_path / "driver.py"
    script.write_text(DRIVER % {"root": ROOT, "lib": lib})
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host checks done" in r.stdout
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
