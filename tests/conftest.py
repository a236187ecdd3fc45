import os
import sys

import pytest


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(autouse=True)
def _trusted_references(request, monkeypatch):
    """Comparison tests take only references the oracle reports as resolved;
    the oracle's own pins look at its raw output."""
    if request.module.__name__.endswith("test_oracle_pins"):
        yield
        return
    import parity
    parity.guard_oracle(monkeypatch)
    yield
