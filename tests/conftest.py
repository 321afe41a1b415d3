import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


def pytest_configure(config):
    import _progress
    _progress._config = config
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through its C ABI)")
    config.addinivalue_line("markers", "slow: runs for minutes on the GPU; only with WL_SLOW_GPU_TESTS=1")


def pytest_collection_modifyitems(config, items):
    import pytest
    if os.environ.get("WL_SLOW_GPU_TESTS") == "1":
        return
    skip = pytest.mark.skip(reason="several minutes on the GPU: set WL_SLOW_GPU_TESTS=1 to run it")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
