import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through its C ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU check")
    config.addinivalue_line("markers", "sanitize: opt-in CPU sanitizer job (BRI_SANITIZE=1)")


@pytest.fixture(scope="session")
def golden_dir():
    return GOLDEN
