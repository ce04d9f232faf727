import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_collection_finish(session):
    # the full-size oracle fits run in forked worker processes from here on, before any test
    # has initialised the GPU
    if any("fullsize_oracle" in getattr(item, "fixturenames", ()) for item in session.items):
        import fullsize_oracle
        fullsize_oracle.start()


def pytest_sessionfinish(session, exitstatus):
    if "fullsize_oracle" in sys.modules:
        sys.modules["fullsize_oracle"].stop()


@pytest.fixture(scope="session")
def fullsize_oracle():
    import fullsize_oracle
    return fullsize_oracle.fit
