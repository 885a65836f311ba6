"""The library's FFT building blocks on the CPU (no GPU): the register
codelets, the four-step composition of every instantiated split and the
generic kernel's Stockham passes against a brute-force DFT, built with g++
under AddressSanitizer and UndefinedBehaviorSanitizer (host-side bounds
checks of every index).  The lists of splits are read from the kernel
sources, so a newly instantiated split is checked automatically."""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_09421_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "cpp")


def _splits():
    """(N_p, N1, N2) of every four-step instantiation in the kernel sources."""
    out = set()
    for f in glob.glob(os.path.join(CSRC, "line4_*.hip")):
        src = open(f).read()
        out |= {(int(a) * int(b), int(a), int(b))
                for a, b in re.findall(r"go_(?:one|long|nw)?<T, (?:true|false|ADJ), (\d+), (\d+)>", src)}
        out |= {(int(a) * int(b), int(a), int(b)) for a, b in re.findall(r"go<T, ADJ, (\d+), (\d+)>", src)}
    return sorted(out)


def _smooth5(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def test_split_table_matches_instantiations():
    src = open(os.path.join(CSRC, "line4_kernels.hip")).read()
    table = {int(np_): (int(a), int(b)) for np_, a, b in
             re.findall(r"case (\d+): \*n1 = (\d+); \*n2 = (\d+); return true;", src)}
    inst = {np_: (a, b) for np_, a, b in _splits()}
    assert table == inst
    assert all(a * b == np_ for np_, (a, b) in table.items())


def test_fft_building_blocks_against_brute_force_dft(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    splits = _splits()
    sizes = sorted({a for _, a, _ in splits} | {b for _, _, b in splits})
    generic = [n for n in range(36, 1201) if _smooth5(n) and n not in {s[0] for s in splits}]
    generic += [90, 288, 540, 1080]   # lengths the generic kernel serves when chosen
    lines = ["CODELET(%d)" % n for n in sizes]
    lines += ["SPLIT(%d, %d)" % (a, b) for _, a, b in splits]
    lines += ["STOCKHAM(%d)" % n for n in generic]
    (tmp_path / "fft_cases.inc").write_text("\n".join(lines) + "\n")
    exe = tmp_path / "fft_check"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", str(tmp_path), "-I", os.path.join(HERE, "stub"), "-I", CSRC,
           os.path.join(HERE, "fft_host_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    m = re.search(r"cases (\d+) failures 0 worst (\S+)", r.stdout)
    assert m and int(m.group(1)) == len(lines), r.stdout[-2000:]
