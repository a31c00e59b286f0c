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
