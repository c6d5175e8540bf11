import os
import sys

import pytest

# Debug guard words for every GPU test: outputs and workspaces allocated by the
# binding's helpers carry a guard zone that is checked after each call.
os.environ.setdefault("MGT_DEBUG", "1")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """Build the host-only libraries (generator, oracle) if they are missing."""
    from workloads import gen
    import oracle
    gen.build(force=False)
    oracle.build(force=False)
    yield
