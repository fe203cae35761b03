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


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of mh_params, mh_request and mh_result have the header's field
    offsets and sizes (compiled with the host C compiler)."""
    import shutil
    import subprocess
    import paper_1407_2737_amd as mh
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"mh_params": mh.Params, "mh_request": mh.Request, "mh_result": mh.Result}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mhkmc.h"',
             "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                        str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for ln in out.splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
