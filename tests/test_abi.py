"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: this runs on machines without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vv10.h")
LIB = os.path.join(ROOT, "paper_2208_14639_amd", "libvv10.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vv10_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for need in ("vv10_prepare", "vv10_energy_potential", "vv10_hessian_terms", "vv10_destroy"):
        assert need in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libvv10.so not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2208_14639_amd import vv10
    for name in declared_functions():
        assert hasattr(vv10, name), name


def test_status_strings_and_version():
    from paper_2208_14639_amd import vv10
    assert vv10.vv10_status_string(0) == "ok"
    assert "not nondecreasing" in vv10.vv10_status_string(-3)
    assert "gfx950" in vv10.vv10_version()


def test_footprint_scales():
    from paper_2208_14639_amd import vv10
    a = vv10.vv10_footprint_bytes(4200, 6, vv10.VV10_FP64)
    b = vv10.vv10_footprint_bytes(27000, 18, vv10.VV10_FP64)
    c = vv10.vv10_footprint_bytes(120000, 60, vv10.VV10_FP64)
    assert 0 < a < b < c
    assert c < 8 * 1024 ** 3          # the 20-mer fits comfortably in 288 GB
    assert vv10.vv10_footprint_bytes(0, 6, 0) == 0
