"""Host-side checks of the C ABI: the library loads, exports every function
include/carve.h declares, and the binding fails loudly without it."""
import ctypes
import os
import re

import pytest

from paper_0901_1307_amd import carve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "carve.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("build_master_index", "scan_image", "flagged_sectors", "confirm_matches"):
        assert n in names
    assert set(names) == set(carve.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(carve.LIB_PATH):
        pytest.skip("libcarve.so is not built")
    lib = ctypes.CDLL(carve.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_match_record_layout():
    assert carve.MATCH_DTYPE.itemsize == 16


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(ImportError):
        carve.load_library(str(tmp_path / "missing.so"))
