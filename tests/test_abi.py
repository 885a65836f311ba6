"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and rejects bad problem descriptions before touching the device.
Also the library's FC table (built in, and its generator) against the
oracle's."""
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


def test_builtin_fc_table_is_the_generated_one():
    """csrc/fc_table_d5_C25.h holds exactly what the committed generator
    writes from fc_tables(5, 25) (hexadecimal doubles, bit for bit)."""
    from paper_2202_09421_amd import gen_fc_table
    assert open(gen_fc_table.OUT).read() == gen_fc_table.render()
    from paper_2202_09421_amd.fc_tables import fc_tables
    Q, A = fc_tables(5, 25)
    vals = [float.fromhex(v) for v in re.findall(r"(-?0x[0-9a-fp.+-]+),", open(gen_fc_table.OUT).read())]
    assert np.array_equal(np.array(vals), np.concatenate([Q.reshape(-1), A.reshape(-1)]))


def _create(prob, beams, nb, dets, nd):
    L = _lib()
    h = ctypes.c_void_p()
    rc = L.rte_plan_create(ctypes.byref(prob), beams, nb, dets, nd, ctypes.byref(h))
    if h.value:
        L.rte_plan_destroy(h)
    return rc, L.rte_last_error().decode()


def test_plan_create_with_null_fc_tables_uses_the_builtin_one():
    """A plain C caller passes no table: validation accepts it for (5, 25);
    without a GPU the call then stops at the device upload."""
    from paper_2202_09421_amd import rte
    prob, beams, nb, dets, nd, keep = _bad_problem()
    assert not prob.fc_Q and not prob.fc_A
    rc, msg = _create(prob, beams, nb, dets, nd)
    assert rc in (rte.RTE_OK, rte.RTE_EDEVICE), msg
    if rc == rte.RTE_EDEVICE:
        assert "upload" in msg
    prob.fc_d = 4
    rc, msg = _create(prob, beams, nb, dets, nd)
    assert rc == rte.RTE_EUNSUPPORTED and "no built-in FC table" in msg


def test_plan_create_rejects_half_a_table_and_unknown_profiles():
    from paper_2202_09421_amd import rte
    prob, beams, nb, dets, nd, keep = _bad_problem()
    Q = (ctypes.c_double * 25)()
    prob.fc_Q = ctypes.cast(Q, ctypes.POINTER(ctypes.c_double))
    rc, msg = _create(prob, beams, nb, dets, nd)
    assert rc == rte.RTE_EINVAL and "together" in msg
    prob, beams, nb, dets, nd, keep = _bad_problem()
    beams[0].profile = 7
    rc, msg = _create(prob, beams, nb, dets, nd)
    assert rc == rte.RTE_EINVAL and "temporal profile" in msg


def test_staged_gradient_argument_checks():
    from paper_2202_09421_amd import rte
    L = _lib()
    n = ctypes.c_int64()
    assert L.rte_gradient_ops(None, ctypes.byref(n)) == rte.RTE_EINVAL
    assert L.rte_gradient_range(None, None, None, None, None, None, None, None, None, 0, 0, 0, None) == rte.RTE_EINVAL
    assert "NULL" in L.rte_last_error().decode()
