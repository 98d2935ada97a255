import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(params=["scalar", "vector"])
def bulk_path(request, monkeypatch):
    """Run a GPU test once per bulk tile shape of the step kernel."""
    monkeypatch.setenv("LBM_BULK_PATH", request.param)
    return request.param
