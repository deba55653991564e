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


def _ensure_built():
    """Builds the oracle and librans when nothing is built yet (the build
    step normally runs first; tests only fill in a missing artefact)."""
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "librans_oracle.so")):
        oracle.build()
    lib = os.path.join(ROOT, "paper_1402_3392_amd", "librans.so")
    if not os.path.exists(lib):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_rans_build", os.path.join(ROOT, "paper_1402_3392_amd", "_build.py"))
        _build = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(_build)
        _build.build()


_ensure_built()
