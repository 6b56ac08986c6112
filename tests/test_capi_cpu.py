"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/fsd.h declares, and its pure-host entry points behave."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    lib = os.path.join(ROOT, "paper_2607_25161_amd", "libfsd.so")
    if not os.path.exists(lib):
        import importlib.util
        spec = importlib.util.spec_from_file_location("_fsd_build", os.path.join(ROOT, "paper_2607_25161_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build(verbose=False)
    import paper_2607_25161_amd as F
    return F


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(fsd_[a-z0-9_]+)\s*\(", src))
    return names


def test_every_declared_symbol_is_exported(F):
    names = _declared()
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(F.lib, n), n


def test_default_params(F):
    p = F.default_params()
    assert p.eta == 1.0 and p.radius == 1.0 and p.r_lub == 3.0 and p.r_precond == 2.1
    assert p.gmres_restart == 30 and p.precision == F.FSD_FP64 and p.lub_eps_min == 1e-3


def test_estimate_bytes_grows_with_size(F):
    p = F.default_params(ewald_tol=1e-5, xi=0.348, grid=128)
    small = F.estimate_bytes(p, 2048, 256, 44.1)
    big = F.estimate_bytes(p, 81920, 4096, 119.7)
    assert 0 < small < big
    assert F.estimate_bytes(p, 0, 1, 10.0) == 0


def test_binding_structs_match_header_layout(F, tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's size and field
    offsets (a small C program built against include/fsd.h prints them)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"fsd_params": F.Params, "fsd_solve_info": F.SolveInfo, "fsd_info": F.Info}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fsd.h"', "int main(void) {"]
    for cname, ct in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in ct._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, field, value = line.split()
        ct = structs[cname]
        want = ctypes.sizeof(ct) if field == "sizeof" else getattr(ct, field).offset
        assert int(value) == want, (cname, field, value, want)
        seen += 1
    assert seen == sum(len(ct._fields_) + 1 for ct in structs.values())
