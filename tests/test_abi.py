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
