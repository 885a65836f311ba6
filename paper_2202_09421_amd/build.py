"""Build the HIP library librte.so (gfx950) in-tree with hipcc.

    python -m paper_2202_09421_amd.build        # or build() from Python
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librte.so")
SOURCES = ["plan.cpp", "capi.cpp", "line_kernels.hip", "line4_kernels.hip", "line4_extra0.hip", "line4_extra1.hip",
           "line4_extra2.hip", "line4_extra3.hip", "line4_long0.hip", "line4_long1.hip", "node_kernels.hip",
           "noalloc.cpp"]
ARCH = os.environ.get("RTE_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    errs = [ln for ln in r.stderr.splitlines() if "warning" in ln and "packed-fp32-ops" not in ln]
    if errs:
        sys.stderr.write("\n".join(errs) + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_sanitized(out_dir: str) -> str:
    """The library with its host code (plan.cpp, capi.cpp) built under
    AddressSanitizer and UndefinedBehaviorSanitizer, linked with the kernel
    objects of the last build(); for CPU tests of the table construction and
    argument checks (load it with the ASan runtime preloaded).  Returns the
    path of the shared library."""
    os.makedirs(out_dir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in SOURCES:
        if src.endswith(".cpp"):
            obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
            cmd = [_hipcc(), "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san + \
                  ["-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr))
        else:
            obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
            if not os.path.exists(obj):
                raise RuntimeError("kernel object %s missing: run build() first" % obj)
        objs.append(obj)
    lib = os.path.join(out_dir, "librte_hostsan.so")
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", lib] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    return lib


if __name__ == "__main__":
    build(verbose=True)
