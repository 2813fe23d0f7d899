import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: long CPU reference computation (opt in with QBE_SLOW=1)")


def pytest_collection_modifyitems(config, items):
    import pytest
    if os.environ.get("QBE_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="long CPU reference run; set QBE_SLOW=1")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
