import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    import oracle as _oracle
    _oracle._load()
    return _oracle


@pytest.fixture(scope="session", autouse=True)
def _library_matches_sources(request):
    """GPU runs test the library built from the sources beside them: a stale
    librdmi.so (built before a source change) is refused before any test."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        from paper_1004_0480_amd import rd
        rd.check_build_matches_sources()
