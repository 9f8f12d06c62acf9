import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")
    # the oracle is compiled here, before any test touches a GPU, if its library is
    # missing or was built from another source (it is never compiled later)
    from oracle import oracle as O
    O.build(force=False)
