"""Host-side checks of the C-ABI library (no GPU needed): it loads, and it
exports every function that include/dgd.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dgd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dgd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dgd_create", "dgd_set_mesh", "dgd_set_material", "dgd_set_state", "dgd_step",
              "dgd_get_seismograms", "dgd_energy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2502_09714_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libdgd.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding's signature table covers the header
    assert set(_declared()) <= set(_lib._SIGS)
