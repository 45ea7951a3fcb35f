import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than ~10 s")


def read_golden(name):
    """Rows of a whitespace-separated fixture under tests/golden, comments dropped."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def hex_bits(h: str, nbits: int) -> int:
    """The first nbits bits of a hex string, as an integer."""
    v = int(h, 16)
    return v >> (4 * len(h) - nbits)


@pytest.fixture(scope="session")
def machin():
    import oracle
    nbits = 100_500
    return nbits, oracle.machin_bits(nbits)


def machin_window(mach, n, w):
    """Bits n .. n+w-1 (1-based) of pi from the Machin bit string."""
    nbits, m = mach
    return (m >> (nbits - (n - 1) - w)) & ((1 << w) - 1)
