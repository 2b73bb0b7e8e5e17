import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running statistical test")


@pytest.fixture(scope="session", autouse=True)
def _built_libraries():
    """Build the oracle (gcc) and the HIP library only if they are not built."""
    import oracle

    oracle.build()
    pkg = os.path.join(ROOT, "paper_1209_0296_amd")
    lib = os.path.join(pkg, "libspinlat.so")
    if os.path.isdir(pkg) and not os.path.exists(lib):
        from paper_1209_0296_amd import build

        build.build(verbose=False)
    yield
