"""The C ABI library loads and exports every entry point that
include/gpsparse.h declares (no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpsparse.h")
LIB = os.path.join(ROOT, "paper_2411_05869_amd", "libgpsparse.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^GP_API\s+[\w\s\*]+?\b(gp_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gp_assemble", "gp_loglik", "gp_predict", "gp_ctx_create", "gp_dataset_create",
                 "gp_matrix_export_csr"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_header():
    from paper_2411_05869_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()
    L = _lib.lib()
    assert L.gp_last_error(None) == b"context is NULL"


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes structures equal those the C
    compiler gives the header's structures."""
    import shutil
    import subprocess
    from paper_2411_05869_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gp_theta": _lib.CTheta, "gp_core": _lib.CCore, "gp_solve_opts": _lib.CSolveOpts,
               "gp_loglik_result": _lib.CLoglikResult, "gp_matrix_layout_info": _lib.CMatrixLayout}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gpsparse.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
