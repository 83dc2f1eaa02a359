"""The Python binding's ctypes signatures against the C declarations (CPU only): every
function of include/pafem.h that the binding binds has the same number of parameters,
each of the matching kind (pointer or handle, int32, int64, size_t, float, double), and
the same kind of result.  A binding that passed a wrong or missing argument would
otherwise fail only on the GPU, or silently."""
import ctypes as C
import os
import re

import pytest

pafem = pytest.importorskip("paper_1911_09220_amd.pafem")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HANDLES = {"pafem_mesh", "pafem_space", "pafem_op", "pafem_net", "pafem_batch", "pafem_pmg"}
SCALARS = {"int32_t": C.c_int32, "pafem_status": C.c_int32, "int64_t": C.c_int64,
           "size_t": C.c_size_t, "float": C.c_float, "double": C.c_double}


def _declarations():
    text = open(os.path.join(ROOT, "include", "pafem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"^(pafem_status|void|int32_t|const char\s*\*)\s*(pafem_\w+)\s*\(([^;]*?)\)\s*;",
                         text, re.M | re.S):
        ret, name, params = m.group(1), m.group(2), " ".join(m.group(3).split())
        plist = [] if params in ("", "void") else [p.strip() for p in params.split(",")]
        out[name] = (ret, plist)
    return out


def _kind_of_param(decl):
    if "*" in decl:
        return "pointer"
    typ = decl.rsplit(" ", 1)[0].replace("const ", "").strip()
    if typ in HANDLES:
        return "pointer"
    return SCALARS[typ]


def _kind_of_ctype(t):
    if t in (C.c_void_p, C.c_char_p) or (isinstance(t, type) and issubclass(t, C._Pointer)):
        return "pointer"
    return t


def test_header_parses_into_every_exported_function():
    decls = _declarations()
    assert len(decls) >= 70
    for name in decls:
        assert hasattr(pafem.lib, name), name


def test_bound_signatures_match_the_header():
    decls = _declarations()
    checked = 0
    for name, (ret, params) in decls.items():
        fn = getattr(pafem.lib, name)
        if fn.argtypes is None:
            continue  # not bound by the Python layer
        checked += 1
        want = [_kind_of_param(p) for p in params]
        got = [_kind_of_ctype(t) for t in fn.argtypes]
        assert got == want, f"{name}: binding {got}, header {want}"
        if ret == "void":
            assert fn.restype is None, name
        elif ret.startswith("const char"):
            assert fn.restype is C.c_char_p, name
        else:
            assert fn.restype is C.c_int32, name
    assert checked >= 60
