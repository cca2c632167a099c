"""The C ABI: the library loads on the CPU host and exports every declared function."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbs.h")
LIB = os.path.join(ROOT, "paper_1709_09347_amd", "libcbs.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cbs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("cbs_apply", "cbs_bicg", "cbs_solve", "cbs_solve_batched", "cbs_grad_vloc",
              "cbs_system_create"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_loads_and_binding_matches_header():
    import paper_1709_09347_amd as cbs
    L = cbs.lib()
    assert sorted(cbs.EXPORTS) == _declared()
    for n in _declared():
        assert hasattr(L, n)
    assert L.cbs_strerror(-4).decode() == "linear solve did not converge"
    p = cbs.default_params()
    assert p.n_q == 32 and p.n_mom == 8 and p.lambda_min == 0.5 and p.tol == 1e-10


def test_struct_layouts_match_header(tmp_path):
    """cbs_params / cbs_info / cbs_grid / cbs_proj: size and every field offset of the
    ctypes mirrors equal what a C compiler makes of include/cbs.h."""
    import ctypes
    import paper_1709_09347_amd as cbs
    structs = {"cbs_params": cbs.Params, "cbs_info": cbs.Info, "cbs_grid": cbs.Grid, "cbs_proj": cbs.Proj}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cbs.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
    assert cbs.default_params().conj_nodes == 1
