"""The C ABI library loads and exports every function include/wf.h declares
(no GPU needed; no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wf.h")
LIB = os.path.join(ROOT, "paper_2501_05938_amd", "libwf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(wf_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_interface():
    names = declared_functions()
    for want in ("wf_init", "wf_destroy", "wf_solve", "wf_solve_batched", "wf_check", "wf_server_create",
                 "wf_submit", "wf_poll", "wf_release", "wf_server_destroy", "wf_last_error", "wf_status_str"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_binding_signatures_cover_header():
    import paper_2501_05938_amd as wf
    lib = wf.load_library()
    assert set(declared_functions()) <= set(wf._SIGS)
    lib.wf_status_str.restype = ctypes.c_char_p
    assert lib.wf_status_str(-5) == b"WF_ETIMEDOUT"
    assert lib.wf_version().startswith(b"libwf")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libwf.so not built")
def test_invalid_arguments_are_rejected_without_a_device_call():
    import paper_2501_05938_amd as wf
    lib = wf.load_library()
    # NULL context and NULL out-pointer are rejected before any HIP call.
    p = wf.Problem()
    assert lib.wf_solve(None, ctypes.byref(p), None) == -1
    assert lib.wf_init(0, None) == -1
    assert lib.wf_check(None) == -1
    assert lib.wf_solve_batched(None, None, 0, None, None) == -1
