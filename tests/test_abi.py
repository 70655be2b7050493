"""The C-ABI library loads and exports every symbol its headers declare
(no GPU needed; no compute calls)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2005_08028_amd", "libscitv.so")


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(sci_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2005_08028_amd import build as hipbuild
        hipbuild.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("sci_forward", "sci_adjoint", "sci_tv_denoise", "sci_gap_tv", "sci_admm_tv"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_null_context_is_rejected_without_a_gpu(lib):
    lib.sci_status_string.restype = ctypes.c_char_p
    assert lib.sci_status_string(-1) == b"invalid argument"

    class Dims(ctypes.Structure):
        _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("B", ctypes.c_int32)]

    f = lib.sci_forward
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, Dims, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert f(None, Dims(4, 4, 2), None, None, None, None) == -1
    lib.sci_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    assert lib.sci_create(None, 0) == -1


def test_binding_raises_when_library_missing(tmp_path):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "scitv_probe", os.path.join(ROOT, "paper_2005_08028_amd", "scitv.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with pytest.raises(RuntimeError):
        mod.load_library(str(tmp_path / "missing.so"))
