"""The C ABI used from plain C: tests/cpp/stream_client.c includes only
include/tstream.h and links only libtstream.so (no Python, no torch in its
process).  It checks STREAM's closed form on the device and on copied-back
elements, a ragged batch run through a captured multi-iteration graph, and
an error status; build() compiles it."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "tests", "cpp", "stream_client")


@pytest.mark.parametrize("n", [1000003, (1 << 24) + 1])
def test_c_client(n):
    assert os.path.exists(CLIENT), "tests/cpp/stream_client is missing: run __graft_entry__.build()"
    print(f"[c client n={n}]", flush=True)
    r = subprocess.run([CLIENT, str(n)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    assert r.stdout.count("ok  ") == 9


def test_ts_log_reports_launch_choices():
    """With TS_LOG set the library names, once per key, the launch
    configuration it picked; without it, it prints nothing."""
    assert os.path.exists(CLIENT), "tests/cpp/stream_client is missing: run __graft_entry__.build()"
    env = dict(os.environ, TS_LOG="1")
    r = subprocess.run([CLIENT, "1000003"], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("tstream: ")]
    for op in ("copy", "scale", "add", "triad"):
        assert any(f"plain {op} f64 n=2^19" in l for l in lines), r.stderr
        assert any(l.startswith(f"tstream: batched {op} f64") for l in lines), r.stderr
    assert len(lines) == len(set(lines))  # once per key
    env.pop("TS_LOG")
    r = subprocess.run([CLIENT, "1000003"], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and "tstream: " not in r.stderr
