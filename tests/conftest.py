import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def paper():
    return golden("paper_numbers.json")


@pytest.fixture(scope="session")
def O():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def acuity(O, paper):
    piv = paper["acuity_pivots"]
    return O.Acuity(piv["ecc_deg"], piv["cpd"])


@pytest.fixture(scope="session")
def layout(O, acuity, paper):
    return O.Layout(acuity, paper["e_max_deg"]["value"])
