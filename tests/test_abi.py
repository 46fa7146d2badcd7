"""The C-ABI library loads and exports every entry point include/slse.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slse.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(slse_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("slse_sketch_apply", "slse_factor", "slse_fused_resid_grad", "slse_solve",
                 "slse_backward", "slse_solve_batched"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2509_06856_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libslse.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(_lib.SIGNATURES) == set(declared_symbols())
    lib2 = _lib.load()
    assert lib2.slse_version().startswith(b"libslse")


def test_struct_layouts_match_header_field_order():
    from paper_2509_06856_amd import _lib

    txt = open(HEADER).read()
    for cls, cname in ((_lib.slse_params, "slse_params"), (_lib.slse_problem, "slse_problem"),
                       (_lib.slse_report, "slse_report"),
                       (_lib.slse_sketch_layout, "slse_sketch_layout")):
        chunk = [c for c in txt.split("typedef struct {") if re.search(r"\}\s*" + cname + ";", c)][0]
        body = chunk[: chunk.index("} " + cname + ";")]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                tok = re.findall(r"[A-Za-z_][A-Za-z_0-9]*", part.split("[")[0])
                names.append(tok[-1])
        assert [f[0] for f in cls._fields_] == names, cname
