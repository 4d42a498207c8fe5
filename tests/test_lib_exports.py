"""The C-ABI library loads on the CPU and exports every symbol include/pf.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("pf_create", "pf_step", "pf_energy", "pf_solute", "pf_adjoint_step", "pf_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2303_09671_amd import pf
    if not os.path.exists(pf.LIB_PATH):
        pytest.skip("libpf.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(pf.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert set(pf.EXPORTS) == set(_declared())


def test_strerror_without_gpu():
    from paper_2303_09671_amd import pf
    if not os.path.exists(pf.LIB_PATH):
        pytest.skip("libpf.so not built")
    assert pf.pf_strerror(pf.PF_EUNSTABLE_DT).startswith("time step")
    assert pf.pf_strerror(pf.PF_ENEGCONC) == "non-positive phase concentration"
