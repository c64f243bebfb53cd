"""The C-ABI library loads and exports every entry point of include/libjacobi.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "libjacobi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jac_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2112_02377_amd import binding
    L = binding.lib()
    names = declared()
    assert "jac_create" in names and "jac_solve_batched" in names and "jac_adjoint" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(binding.EXPORTS) == names


def test_status_strings_are_host_only():
    from paper_2112_02377_amd import binding
    assert binding.status_name(0) == "JAC_OK"
    assert binding.status_name(-6) == "JAC_E_DIVERGED"
    assert binding.status_name(1) == "JAC_NOT_CONVERGED"
