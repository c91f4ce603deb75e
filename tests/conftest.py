import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) HIP device")


import json

import pytest


@pytest.fixture(scope="session")
def golden_tables():
    with open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")) as fh:
        return json.load(fh)
