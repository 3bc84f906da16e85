"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point declared in include/raks.h, and reports a missing device
as RAKS_EDEVICE rather than crashing."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "raks.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(raks_\w+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("raks_create", "raks_destroy", "raks_load_graph", "raks_query",
                 "raks_query_batch", "raks_results_free", "raks_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2001_06770_amd as raks
    if not os.path.exists(raks.LIB_PATH):
        from paper_2001_06770_amd import build
        build.build()
    lib = ctypes.CDLL(raks.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(raks.EXPORTED) == set(declared())
    lib.raks_version.restype = ctypes.c_char_p
    assert lib.raks_version().startswith(b"raks-gfx950")


def test_no_device_is_an_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2001_06770_amd as raks
    with pytest.raises(raks.RaksError) as e:
        raks.Context(0, use_torch=False)
    assert e.value.code == -3


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2001_06770_amd as raks
    monkeypatch.setattr(raks, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(raks, "_lib_handle", None)
    with pytest.raises(RuntimeError):
        raks.lib()


LAYOUT_STRUCTS = {
    "raks_ctx_opts": "CtxOpts", "raks_serve_opts": "ServeOpts", "raks_graph_desc": "GraphDesc",
    "raks_query_desc": "QueryDesc", "raks_arc": "Arc", "raks_result": "Result",
    "raks_query_stats": "QueryStats", "raks_results": "Results",
    "raks_kernel_timing": "KernelTiming", "raks_tuning": "Tuning",
    "raks_results_buf": "ResultsBuf",
}


def test_binding_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the C compiler's sizes and
    field offsets (a mismatch would corrupt every call silently)."""
    import paper_2001_06770_amd as raks
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "raks.h"', "int main(void) {"]
    for cname, pyname in LAYOUT_STRUCTS.items():
        st = getattr(raks, pyname)
        lines.append(f'printf("{pyname} size %zu\\n", sizeof({cname}));')
        for fname, _ in st._fields_:
            lines.append(f'printf("{pyname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    for line in filter(None, out):
        pyname, field, value = line.split()
        st = getattr(raks, pyname)
        got = ctypes.sizeof(st) if field == "size" else getattr(st, field).offset
        assert got == int(value), (pyname, field, got, value)
