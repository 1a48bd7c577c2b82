"""The C ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_1104_2732_amd", "libcpselect.so")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;",
                             text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "return", "sizeof"):
                names.append(name)
    return names


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("select_kth", "select_kth_ex", "cps_objective", "cps_create", "cps_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_checks_and_strings():
    import paper_1104_2732_amd as cps
    L = cps.lib()
    assert L.cps_status_string(0) == b"ok"
    assert L.cps_status_string(-1) == b"invalid argument"
    o = cps.default_options()
    assert o.maxit == 64 and o.final_threshold > 0 and 0 < o.partition_fraction <= 1
    # null handle / bad sizes are rejected before any device work
    out = ctypes.c_void_p(0)
    assert L.select_kth(None, None, 10, 1, 0, out, None) == -1
    assert L.select_kth_ex(None, ctypes.c_void_p(16), 0, 1, 0, None, out, None, None) == -1
    assert L.cps_objective(None, ctypes.c_void_p(16), 10, 11, 0, None, 1, out, None) == -1
    assert L.cps_destroy(None) == -1
