import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_addoption(parser):
    parser.addoption("--shk-tune", default="",
                     help="knob=value,... applied to the library's shared tuning settings for the session")


@pytest.fixture(autouse=True, scope="session")
def _shk_tune_session(request):
    spec = request.config.getoption("--shk-tune")
    if not spec:
        yield
        return
    import paper_1212_3660_amd as P
    for kv in spec.split(","):
        k, v = kv.split("=")
        P.shk_tune_set(P.TUNE_ALL, k.strip(), float(v))
    yield
    P.shk_tune_reset()
