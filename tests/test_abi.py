"""Host-side checks of the C ABI: the library loads and exports every symbol the
header declares; without a GPU, context creation fails cleanly."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gw.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gw_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    names = header_functions()
    for n in ("gw_mtxel_spinor", "gw_chi0_accumulate", "gw_epsinv", "gw_chi0_closure"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2206_00808_amd.binding as B
    lib = B.raw()
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(B.EXPORTED) == header_functions()


def test_status_strings():
    import paper_2206_00808_amd as P
    assert P.status_string(P.GW_EALIAS) == "GW_EALIAS"
    assert P.status_string(P.GW_ESINGULAR) == "GW_ESINGULAR"
    assert P.status_string(P.GW_EFALLBACK) == "GW_EFALLBACK"


def test_context_without_device_reports_edevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    import paper_2206_00808_amd as P
    with pytest.raises(P.GwError) as ei:
        P.Context(0)
    assert ei.value.status == P.GW_EDEVICE


def test_header_compiles_as_c():
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        with open(src, "w") as f:
            f.write('#include "gw.h"\nint main(void){gw_ctx* c=0; (void)c; return 0;}\n')
        r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                            src, "-o", os.path.join(d, "t")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
