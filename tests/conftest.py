import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: minutes of oracle work; runs only with WTD_SLOW_TESTS=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("WTD_SLOW_TESTS") == "1":
        return
    skip = pytest.mark.skip(reason="minutes of oracle work; set WTD_SLOW_TESTS=1 to run")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def systems():
    """Cache of seeded synthetic systems keyed by config name."""
    from gen import CONFIGS, make_system
    cache = {}

    def get(name, **over):
        key = (name, tuple(sorted(over.items())))
        if key not in cache:
            cache[key] = make_system(CONFIGS[name], **over)
        return cache[key]

    return get
