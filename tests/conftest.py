import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def codec16():
    from paper_1404_3458_amd import rs

    c = rs.Codec(16)
    yield c
    c.close()


@pytest.fixture(scope="session")
def codec8():
    from paper_1404_3458_amd import rs

    c = rs.Codec(8)
    yield c
    c.close()
