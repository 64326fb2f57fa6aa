import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionstart(session):
    """Build the library and the C client when nothing is built yet (a fresh
    checkout); an existing build is used as it is."""
    lib = os.path.join(ROOT, "paper_2206_06302_amd", "libtstream.so")
    client = os.path.join(ROOT, "tests", "cpp", "stream_client")
    if os.path.exists(lib) and os.path.exists(client):
        return
    import __graft_entry__ as entry

    if not os.path.exists(lib):
        entry._load_build_module().build(verbose=True)
    entry.build_c_client()


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build(force=False)
    return oracle
