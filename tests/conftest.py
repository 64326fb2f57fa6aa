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
    """Build the library when it is missing or older than any of its sources,
    and the C client when it is missing or older than its source or the
    library, so the tests always run the sources of this tree."""
    import __graft_entry__ as entry

    lib = os.path.join(ROOT, "paper_2206_06302_amd", "libtstream.so")
    client = os.path.join(ROOT, "tests", "cpp", "stream_client")
    client_src = client + ".c"
    builder = entry._load_build_module()
    if builder.stale():
        builder.build(verbose=True)
    if (not os.path.exists(client) or os.path.getmtime(client) < os.path.getmtime(client_src)
            or os.path.getmtime(client) < os.path.getmtime(lib)):
        entry.build_c_client()


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build(force=False)
    return oracle
