"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function that
include/gpe.h declares, and rejects invalid problems before touching the device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "gpe.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gpe_[A-Za-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def gpe():
    from paper_1611_02045_amd import gpe as mod
    if not os.path.exists(mod.LIB_PATH):
        pytest.skip("libgpe.so not built")
    mod.lib()
    return mod


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ("gpe_energy", "gpe_apply_H", "gpe_precond", "gpe_pcg_solve", "gpe_plan_create",
                     "gpe_pcg_solve_batched", "gpe_energy_grad", "gpe_adjoint_solve", "gpe_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(gpe):
    L = ctypes.CDLL(gpe.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, f"symbols declared in gpe.h but not exported: {missing}"
    # and the binding covers all of them
    assert set(_declared_functions()) <= set(gpe.SIGNATURES)


def test_struct_layouts_match_header(gpe, tmp_path):
    """The ctypes mirrors have the sizes and field offsets the C compiler gives the header."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gpe_problem_t": gpe.Problem, "gpe_pcg_opts_t": gpe.PcgOpts, "gpe_pcg_report_t": gpe.PcgReport}
    rename = {"lam": "lambda"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gpe.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            cf = rename.get(fname, fname)
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.split("\n") if line)
    for cname, cls in structs.items():
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


@pytest.mark.parametrize("dim,n,L,omega,status", [
    (4, (8, 8, 8), (1, 1, 1), 0.0, -1),        # bad dimension
    (2, (12, 8), (1, 1), 0.0, -2),             # not a power of two
    (2, (7, 8), (1, 1), 0.0, -1),              # odd
    (1, (16,), (1,), 0.5, -1),                 # rotation in 1-D
    (2, (16, 16), (1.0, -1.0), 0.0, -1),       # negative half-width
    (2, (2048, 8), (1.0, 1.0), 0.0, -2),       # too large
])
def test_invalid_problems_are_rejected_on_the_host(gpe, dim, n, L, omega, status):
    prob = gpe.make_problem(dim, n, L, 1.0, omega)
    h = ctypes.c_void_p()
    st = gpe.lib().gpe_plan_create(ctypes.byref(prob), 0, ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert len(gpe.lib().gpe_last_error()) > 0


def test_default_options(gpe):
    o = gpe.default_opts()
    assert o.method == 1 and o.precond == 3 and o.tol_res_inf == 1e-8
    o = gpe.default_opts(precond="kinetic", method="pg", precision="mixed")
    assert (o.precond, o.method, o.precision) == (1, 0, 1)
