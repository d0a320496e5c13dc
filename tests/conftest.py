import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs (set WV_SLOW=1 to run)")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("WV_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow oracle pin; set WV_SLOW=1")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


def read_golden(name):
    """Rows of a whitespace-separated fixture under tests/golden, comments dropped."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows
