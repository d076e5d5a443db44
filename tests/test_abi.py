"""The C ABI library loads and exports every entry point declared in include/vms.h (not gpu).

No compute call is made: loading the shared object needs no device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vms.h")
LIB = os.path.join(ROOT, "paper_0809_4802_amd", "libvms.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vms_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for required in ("vms_element_tangents", "vms_condense_assemble", "vms_newton_step", "vms_gmres_solve",
                     "vms_create", "vms_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvms.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvms.so not built")
def test_binding_covers_the_header():
    import sys
    sys.path.insert(0, ROOT)
    src = open(os.path.join(ROOT, "paper_0809_4802_amd", "binding.py")).read()
    exported = re.search(r"EXPORTED = \[(.*?)\]", src, flags=re.S).group(1)
    listed = sorted(re.findall(r'"(vms_[a-z0-9_]+)"', exported))
    assert listed == declared_functions()


def test_last_error_without_context():
    if not os.path.exists(LIB):
        pytest.skip("libvms.so not built")
    lib = ctypes.CDLL(LIB)
    lib.vms_create.restype = ctypes.c_int
    lib.vms_last_error.restype = ctypes.c_char_p
    lib.vms_last_error.argtypes = [ctypes.c_void_p]
    # NULL out-pointer is rejected on the host before any device call
    rc = lib.vms_create(None, None, None, None)
    assert rc == -1
    assert b"NULL" in lib.vms_last_error(None)
