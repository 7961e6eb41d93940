"""Host-side checks of the HIP library that need no GPU: the generated
Marching Cubes table, the exported C ABI, and the binding's failure modes."""
import ctypes
import importlib.util
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_08475_amd", "csrc")
HEADER = os.path.join(ROOT, "include", "amriso.h")
LIB = os.path.join(ROOT, "paper_2004_08475_amd", "libamriso.so")


def _table_from_inc():
    txt = open(os.path.join(CSRC, "mc_table.inc")).read()
    words = [int(w, 16) for w in re.findall(r"0x([0-9a-f]{16})ull", txt)]
    assert len(words) == 256
    return words


def test_gpu_table_equals_oracle_polygonisation():
    """The GPU table (written by its own generator) encodes exactly the
    oracle's procedural polygonisation, case by case and triangle by triangle."""
    for case, w in enumerate(_table_from_inc()):
        nt = w >> 60
        tris = [tuple((w >> (12 * t + 4 * v)) & 0xF for v in range(3)) for t in range(nt)]
        want = [tuple(int(e) for e in r) for r in oracle.polygonize(case)]
        assert tris == want, case


def test_committed_table_is_generator_output():
    spec = importlib.util.spec_from_file_location("mc_table_gen", os.path.join(CSRC, "mc_table_gen.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert mod.render() == open(os.path.join(CSRC, "mc_table.inc")).read()


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(amr_\w+)\s*\(", txt, re.M)))


def test_header_declares_binding_symbols():
    import paper_2004_08475_amd as amr

    assert _declared() == sorted(amr.ABI_SYMBOLS)


def test_library_loads_and_exports_abi():
    if not os.path.exists(LIB):
        pytest.fail("libamriso.so missing: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    for sym in _declared():
        assert getattr(lib, sym, None) is not None, sym
    lib.amr_last_error.restype = ctypes.c_char_p
    assert lib.amr_last_error() == b""


def test_binding_null_arguments_are_errors():
    import paper_2004_08475_amd as amr

    lib = amr.load_library()
    assert lib.amr_create(None, 0) == amr.AMR_EINVAL
    assert b"NULL" in lib.amr_last_error()
    assert lib.amr_upload(None, None, None, None, 0, None) == amr.AMR_EINVAL
    assert lib.amr_isosurface(None, ctypes.c_float(0.0), None, None, None, 0, None, None) == amr.AMR_EINVAL
    sz = ctypes.c_size_t(0)
    assert lib.amr_index_bytes(None, ctypes.byref(sz)) == amr.AMR_EINVAL
    lib.amr_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_2004_08475_amd as amr

    saved = amr._lib
    try:
        amr._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            amr.load_library(str(tmp_path / "missing.so"))
    finally:
        amr._lib = saved


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2004_08475_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".inc", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), f
                assert "amr_oracle" not in txt and "liborc" not in txt, f
