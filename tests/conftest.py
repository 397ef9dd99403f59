import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def tiny_keys():
    import oracle
    import seeded_inputs as si
    return oracle.Keys(si.TINY, si.KEY_SEED_BASE + 100)


@pytest.fixture(scope="session")
def toy_keys():
    import oracle
    import seeded_inputs as si
    return oracle.Keys(si.TOY, si.KEY_SEED_BASE + 1)
