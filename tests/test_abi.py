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


def test_info_struct_and_enums_match_the_header(tmp_path):
    # compile a probe against the header with the host C compiler: the ctypes
    # mirror of jac_info must have the same size and field offsets, and the
    # binding's option and status numbers must equal the header's enums
    import subprocess
    from paper_2112_02377_amd import binding
    fields = [f for f, _ in binding.jac_info._fields_]
    opts = [n for n in dir(binding) if n.startswith("JAC_OPT_")]
    stats = ["JAC_OK", "JAC_NOT_CONVERGED", "JAC_E_INVALID", "JAC_E_ZERO_DIAG", "JAC_E_NOMEM", "JAC_E_HIP",
             "JAC_E_STATE", "JAC_E_DIVERGED", "JAC_BANDROW", "JAC_BANDROW_SP", "JAC_SUBSTRUCT",
             "JAC_NORM_L2_REL", "JAC_NORM_INF_ABS", "JAC_FP64", "JAC_FP32_REFINE"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "libjacobi.h"', "int main(void) {",
             '  printf("size %zu\\n", sizeof(jac_info));']
    lines += [f'  printf("off {f} %zu\\n", offsetof(jac_info, {f}));' for f in fields]
    lines += [f'  printf("enum {e} %d\\n", (int){e});' for e in opts + stats]
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            kind, *rest = line.split()
            got[(kind, rest[0] if len(rest) > 1 else "")] = int(rest[-1])
    assert got[("size", "")] == ctypes.sizeof(binding.jac_info)
    for f in fields:
        assert got[("off", f)] == getattr(binding.jac_info, f).offset, f
    for e in opts + stats:
        assert got[("enum", e)] == getattr(binding, e), e
