"""The C-ABI library loads and exports every function include/fvem.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fvem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fvem_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fvem_hierarchy_build", "fvem_solve", "fvem_solve_adjoint", "fvem_hierarchy_destroy",
              "fvem_last_error", "fvem_apply"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2607_17725_amd import fvem
    if not os.path.exists(fvem.LIB_PATH):
        pytest.skip("libfvem.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(fvem.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(fvem.EXPORTS) == set(_declared())


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2607_17725_amd import fvem
    with pytest.raises(fvem.FvemError):
        fvem._lib = None
        fvem.load(str(tmp_path / "missing.so"))
