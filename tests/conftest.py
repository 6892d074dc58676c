import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def soe_tables():
    from oracle import soe
    t = {M: soe.load_table(os.path.join(GOLDEN, "soe_talbot_M%d.txt" % M))
         for M in (8, 12, 16, 20, 24)}
    # model-reduced table (balanced truncation), keyed by name
    t["r10"] = soe.load_table(os.path.join(GOLDEN, "soe_reduced_M10.txt"))
    return t
