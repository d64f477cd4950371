"""The C-ABI library loads and exports every function include/th.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os

import pytest

from paper_2509_17494_amd import _lib as L


def test_header_declares_the_entry_points():
    names = L.declared_functions()
    for n in ["th_setup_fine", "th_setup_coarse", "th_smooth", "th_residual", "th_restrict",
              "th_prolong", "th_solve", "th_create", "th_destroy", "th_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libth.so is not built (run `python -m paper_2509_17494_amd.build`)")
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in L.declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    lib = L.load()
    for n in L.declared_functions():
        assert getattr(lib, n).restype is not None or n.endswith("_destroy"), n
