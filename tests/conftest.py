import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(params=["auto", "pairs", "pairs_held", "single-scalar", "single-vector"])
def schedule(request, monkeypatch):
    """Run a GPU test once per kernel schedule of lbm_step, chosen through
    lbm_params: the default (three steps per launch with the Zou & He
    outflow at FP32 and FP16, two otherwise), two steps per launch (the
    walk chosen by lattice size, and the walk that holds a row's stores
    back, forced; it has no FP16 form), and one step per launch with each
    bulk tile shape."""
    from paper_2506_05293_amd import lbm
    launch, _, path = request.param.partition("-")
    monkeypatch.setitem(lbm.LATTICE_DEFAULTS, "launch", launch)
    monkeypatch.setitem(lbm.LATTICE_DEFAULTS, "bulk_path", path or "auto")
    return request.param
