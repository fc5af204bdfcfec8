"""The C-ABI library loads and exports every symbol include/dd.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd.h")
LIB = os.path.join(ROOT, "paper_2109_05908_amd", "libdd.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for f in ("dd_setup", "dd_apply", "dd_pcg", "dd_info", "dd_destroy", "dd_partition_ggg", "dd_gmres",
              "dd_setup_batch", "dd_update_values", "dd_trim_device_cache"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_binding_signatures_cover_header():
    from paper_2109_05908_amd.binding import exported_symbols
    assert set(declared_functions()) <= set(exported_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdd.so not built")
def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.dd_strerror.restype = ctypes.c_char_p
    assert lib.dd_strerror(0) == b"ok"
    assert b"SPD" in lib.dd_strerror(-2)


def test_binding_constants_equal_header_defines():
    """Every numeric #define of the header that the binding mirrors has the same value there."""
    import paper_2109_05908_amd.binding as B
    src = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(DD_[A-Z0-9_]+)\s+(-?\d+)\b", src)}
    mirrored = [k for k in defs if hasattr(B, k)]
    assert len(mirrored) >= 20
    for k in mirrored:
        assert getattr(B, k) == defs[k], k
