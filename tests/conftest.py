import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_core():
    from oracle import core
    core.lib()
    return core


@pytest.fixture(scope="module")
def reading_blob_module():
    """The oracle's kernel functions use the blob of the kernel reading (not
    its default, the paper's blob) for the whole module: modules that pin
    that kernel, or run the oracle's forward model at sizes where the paper
    blob's per-pair quadrature would take hours."""
    from oracle import core
    with core.reading_blob():
        yield
