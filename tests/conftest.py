import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


@pytest.fixture(scope="session")
def inst13():
    from opfgen import build_instance, make_13bus
    return build_instance(make_13bus(0))


@pytest.fixture(scope="session")
def inst13zip():
    from opfgen import build_instance, make_13bus
    return build_instance(make_13bus(0, zip_variant=True))


@pytest.fixture(scope="session")
def inst123():
    from opfgen import build_instance, make_123bus
    return build_instance(make_123bus(0))
