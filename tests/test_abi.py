"""The C ABI library loads and exports every function include/ccpt.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccpt.h")
LIB = os.path.join(ROOT, "paper_2310_08770_amd", "libccpt.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccpt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared()
    for required in ("ccpt_set_reference", "ccpt_track_batch", "ccpt_track_grad", "ccpt_create",
                     "ccpt_destroy", "ccpt_fisher"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libccpt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libccpt.so not built")
def test_binding_covers_every_export():
    from paper_2310_08770_amd.ccpt import EXPORTS
    assert sorted(EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libccpt.so not built")
def test_host_only_calls():
    lib = ctypes.CDLL(LIB)
    lib.ccpt_status_string.restype = ctypes.c_char_p
    assert lib.ccpt_status_string(0) == b"ok"
    assert lib.ccpt_status_string(-2) == b"unsupported frame size"
    # null context arguments are rejected without touching a device
    assert lib.ccpt_track_batch(None, None, 0, None, None) == -1
    assert lib.ccpt_create(None, 0, None) == -1
