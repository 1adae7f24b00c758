import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Compile the C oracle once per session (it is test infrastructure)."""
    import oracle

    src = os.path.join(ROOT, "oracle", "ppml_oracle.c")
    lib = oracle.lib_path()
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        oracle.build()
    yield
