"""The C-ABI library builds, loads and exports every entry point that
include/ffbie.h declares (no GPU needed; no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ffbie.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ffbie_status|const char \*|int64_t|int)\s*(ffbie_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    assert "ffbie_kernel_coeffs" in names and "ffbie_create" in names
    assert len(names) >= 6


def test_library_exports_every_declared_symbol():
    import paper_2608_16208_amd as ffbie
    if not os.path.exists(ffbie.LIB_PATH):
        from paper_2608_16208_amd import build
        build.build()
    lib = ctypes.CDLL(ffbie.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(ffbie.EXPORTS)


def test_errors_without_gpu_work():
    """Argument checks that return before any device work."""
    import paper_2608_16208_amd as ffbie
    lib = ffbie.load_library()
    assert lib.ffbie_destroy(None) == 0
    assert lib.ffbie_last_error(None)
    assert lib.ffbie_create(None, 0, None) == -1
