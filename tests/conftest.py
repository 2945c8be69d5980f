import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (gfx950) and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _built_library():
    """Builds the HIP library once if no build is present (the library is
    never rebuilt over an existing one here)."""
    from paper_1507_03521_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1507_03521_amd import build
        build.build()
    yield
