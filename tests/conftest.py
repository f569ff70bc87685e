import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long statistical test")


@pytest.fixture(scope="session")
def orc():
    from oracle import su2_oracle
    su2_oracle._load()
    return su2_oracle


@pytest.fixture(scope="session")
def su2():
    """The GPU library through its Python binding (fails loudly if not built)."""
    import paper_1010_1486_amd as pkg
    return pkg
