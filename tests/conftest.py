import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built librans")
    config.addinivalue_line("markers", "slow: long-running (full-size workloads)")


def load_golden(name):
    """Parses a 'key v1 v2 ...' text fixture under tests/golden/."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = [int(v) for v in vals]
    return out


@pytest.fixture(scope="session")
def golden_example():
    return load_golden("worked_example.txt")
