import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-scale case (minutes of CPU oracle time)")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_helpers():
    """The workload sampler and the oracle are plain C; build them when absent."""
    import oracle
    import workload
    workload.build(force=False)
    oracle.build(force=False)
    yield
