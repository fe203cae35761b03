"""The C-ABI library loads and exports every symbol that include/mhkmc.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhkmc.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mh_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("mh_create_assembly", "mh_run_loops", "mh_get_loop", "mh_get_sar",
                 "mh_run_batch"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1407_2737_amd as mh
    if not os.path.exists(mh.LIB_PATH):
        from paper_1407_2737_amd import build
        build.build()
    lib = ctypes.CDLL(mh.LIB_PATH)
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(mh.SYMBOLS) == set(_declared())


def test_error_strings_without_device():
    import paper_1407_2737_amd as mh
    L = mh._lib()
    assert L.mh_strerror(0) == b"ok"
    assert L.mh_strerror(-2) == b"particles overlap"
    # no device here: creating a context must fail cleanly, not crash
    h = ctypes.c_void_p()
    rc = L.mh_ctx_create(99, ctypes.byref(h))
    assert rc == -4 and not h.value
