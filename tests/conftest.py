import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libjacobi.so")
    config.addinivalue_line("markers", "slow: large CPU case (still part of the default CPU suite)")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def read_golden(name):
    """Parse a whitespace golden file into {key: [token lists]} (comments '#')."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            out.setdefault(key, []).append(rest)
    return out


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import ref
    return ref.lib()
