import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # run the oracle pins first, GPU parity afterwards, and anything named test_zz_* last
    def rank(item):
        name = item.fspath.basename
        if name.startswith("test_zz_"):
            return 2
        return 1 if item.get_closest_marker("gpu") else 0
    items.sort(key=rank)


@pytest.fixture(scope="session")
def ora():
    import oracle
    oracle.lib()
    return oracle
