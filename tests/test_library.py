"""The C-ABI library (CPU only: no GPU calls): it loads, exports every
function that include/sn.h declares, and the Python binding wraps exactly
that set.  sn_inflow_size is pure host arithmetic and is checked against
the input module's boundary layout."""
import ctypes
import os
import re
import shutil

import pytest

import sninputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sn.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)      # drop comments
    text = re.sub(r"//[^\n]*", " ", text)
    names = re.findall(r"(?:^|;|\})\s*(?:const\s+)?\w[\w\s\*]*?\b(sn_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def library():
    from paper_2001_09196_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
            pytest.skip("libsn.so not built and no hipcc")
        from paper_2001_09196_amd import build
        build.build()
    return ctypes.CDLL(binding.LIB_PATH), binding


def test_header_parses():
    names = header_functions()
    assert "sn_sweep" in names and "sn_source_iterate" in names and "sn_last_error" in names
    assert len(names) >= 13


def test_exports_match_header():
    lib, binding = library()
    names = header_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared in sn.h but not exported: {missing}"
    assert sorted(binding.EXPORTED) == names


def test_inflow_size_host_logic():
    lib, binding = library()
    for dim, nx, ny, nz in ((2, 16, 9, 1), (3, 7, 5, 3), (3, 128, 128, 128)):
        m = binding.sn_mesh(dim, nx, ny, nz, 1.0, 1.0, 1.0)
        assert binding.lib().sn_inflow_size(ctypes.byref(m)) == sninputs.inflow_size(dim, nx, ny, nz)
    for order in (2, 3, 4):                    # order p: (p + 1) values per boundary face
        m = binding.sn_mesh(2, 16, 9, 1, 1.0, 1.0, 1.0, order)
        assert binding.lib().sn_inflow_size(ctypes.byref(m)) == (order + 1) * (16 + 9)
