"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and rejects bad problem descriptions before touching the device.
Also the library's host-side FC table builder against the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rte.h")).read()
    return sorted(set(re.findall(r"\b(rte_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_2202_09421_amd import rte
    if not os.path.exists(rte.LIB_PATH):
        from paper_2202_09421_amd.build import build
        build()
    return rte.lib()


def test_every_declared_symbol_is_exported():
    L = _lib()
    names = _declared()
    assert {"rte_plan_create", "rte_forward", "rte_adjoint", "rte_gradient"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def _bad_problem(**kw):
    import workloads as W
    from paper_2202_09421_amd import rte
    spec = W.small_problem(N=12, M=8, K=4)
    prob, beams, nb, dets, nd, keep = rte.make_problem(spec)
    for k, v in kw.items():
        setattr(prob, k, v)
    return prob, beams, nb, dets, nd, keep


@pytest.mark.parametrize("field,value,msg", [
    ("M", 6, "multiple of 4"),
    ("Nx", 5, "2*fc_d"),
    ("K", 0, "K must"),
    ("g", 1.0, "|g|"),
    ("dt", -1.0, "dt and c"),
    ("dtype", 7, "dtype"),
    ("dt", 50.0, "AB4 stability limit"),
])
def test_plan_create_rejects_bad_input(field, value, msg):
    from paper_2202_09421_amd import rte
    L = _lib()
    prob, beams, nb, dets, nd, keep = _bad_problem(**{field: value})
    h = ctypes.c_void_p()
    rc = L.rte_plan_create(ctypes.byref(prob), beams, nb, dets, nd, ctypes.byref(h))
    assert rc == rte.RTE_EINVAL
    assert msg in L.rte_last_error().decode()
    assert not h.value


@pytest.mark.parametrize("what", ["beam", "detector"])
def test_plan_create_rejects_sources_off_the_boundary(what):
    from paper_2202_09421_amd import rte
    L = _lib()
    prob, beams, nb, dets, nd, keep = _bad_problem()
    arr = beams if what == "beam" else dets
    arr[0].x, arr[0].y = 0.5 * (prob.xmin + prob.xmax), 0.5 * (prob.ymin + prob.ymax)
    h = ctypes.c_void_p()
    assert L.rte_plan_create(ctypes.byref(prob), beams, nb, dets, nd, ctypes.byref(h)) == rte.RTE_EINVAL
    assert "%s 0 is not on the boundary" % what in L.rte_last_error().decode()
    assert not h.value


def test_null_arguments_are_errors():
    from paper_2202_09421_amd import rte
    L = _lib()
    assert L.rte_plan_create(None, None, 0, None, 0, None) == rte.RTE_EINVAL
    assert L.rte_forward(None, None, None, None, None, 0, None, 0, None) == rte.RTE_EINVAL
    assert "NULL" in L.rte_last_error().decode()
    assert L.rte_adjoint(None, None, None, None, None, None, None, 0, None) == rte.RTE_EINVAL
    assert L.rte_plan_set_guard(None, 1) == rte.RTE_EINVAL


def test_library_fc_tables_match_oracle():
    from oracle.fc_gram import blend_table
    from paper_2202_09421_amd.fc_tables import fc_tables
    Q, A = fc_tables(5, 25)
    Qo, Ao = blend_table(5, 25)
    assert np.allclose(Q, Qo, rtol=0, atol=1e-15)
    assert np.allclose(A, Ao, rtol=1e-14, atol=1e-14 * np.abs(Ao).max())


def test_binding_struct_layouts_match_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the header's struct of the same name."""
    import shutil
    import subprocess
    from paper_2202_09421_amd import rte
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [rte.rte_problem, rte.rte_beam, rte.rte_detector, rte.rte_schedule, rte.rte_separable,
               rte.rte_forward_extra]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rte.h"', "int main(void) {"]
    for S in structs:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (S.__name__, S.__name__))
        for f in S._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (S.__name__, f[0], S.__name__, f[0]))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for S in structs:
        assert int(got[S.__name__]) == ctypes.sizeof(S), S.__name__
        for f in S._fields_:
            assert int(got["%s.%s" % (S.__name__, f[0])]) == getattr(S, f[0]).offset, (S.__name__, f[0])
