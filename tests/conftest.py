"""Test configuration: the ``gpu`` marker and shared helpers.

Tests marked ``gpu`` need an MI355X (gfx950) and the built HIP library; every
other test runs on the CPU.  The CPU oracle is test infrastructure and is
(re)built here with g++ if its shared library is missing.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    from oracle import build as obuild
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH) or os.path.getmtime(O.LIB_PATH) < os.path.getmtime(obuild.SRC):
        obuild.build()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.lib()
    return O
