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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libccpt.so not built")
@pytest.mark.parametrize("rate_limit", [0.0, 0.005])
def test_drift_filter_matches_the_oracle(rate_limit):
    """ccpt_drift_filter is host code: the same stream in one call and in
    three pieces (state carried) against the oracle's Eq. 10-12."""
    import numpy as np
    from oracle import ccpt_oracle as O
    from paper_2310_08770_amd import drift_filter
    rng = np.random.Generator(np.random.PCG64(3))
    r = np.cumsum(rng.normal(0, 0.2, size=(300, 2)), axis=0) + 0.5
    _, want = O.drift_filter(r, 0.05, rate_limit)
    got, _ = drift_filter(r, 0.05, rate_limit)
    assert np.max(np.abs(got - want)) <= 1e-12
    st = None
    parts = []
    for a, b in ((0, 70), (70, 71), (71, 300)):
        p, st = drift_filter(r[a:b], 0.05, rate_limit, st)
        parts.append(p)
    assert np.max(np.abs(np.vstack(parts) - want)) <= 1e-12


@pytest.mark.skipif(not os.path.exists(LIB), reason="libccpt.so not built")
def test_drift_filter_rejects_bad_arguments():
    lib = ctypes.CDLL(LIB)
    lib.ccpt_drift_filter.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    st = (ctypes.c_double * 3)()
    assert lib.ccpt_drift_filter(None, 3, 0.1, 0.0, st, None) == -1
    assert lib.ccpt_drift_filter(None, 0, 1.5, 0.0, st, None) == -1
    assert lib.ccpt_drift_filter(None, 0, 0.1, -1.0, st, None) == -1
    st[2] = -1.0
    assert lib.ccpt_drift_filter(None, 0, 0.1, 0.0, st, None) == -1
