"""The GPU-free host code under the compilers' sanitizers (CPU only): the
oracle under AddressSanitizer + UndefinedBehaviorSanitizer and, for its
threaded timed mode, ThreadSanitizer; the library's tuning-file parser,
planners and pinned worker pool likewise.  Any report fails the test
(-fno-sanitize-recover, halt_on_error)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2206_06302_amd", "csrc")
HOST_SOURCES = [os.path.join(ROOT, "tests", "cpp", "san_host.cpp"), os.path.join(CSRC, "tune.cpp"),
                os.path.join(CSRC, "host_target.cpp")]
ORACLE_SOURCES = [os.path.join(ROOT, "tests", "cpp", "san_oracle.c"), os.path.join(ROOT, "oracle", "oracle.c")]
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1",
           TSAN_OPTIONS="halt_on_error=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _build(tmp_path, cc, std, flags, sources, includes, name):
    out = tmp_path / name
    cmd = [cc, std, "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-sanitize-recover=all",
           *flags, *("-I" + i for i in includes), "-o", str(out), *sources, "-lpthread", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return str(out)


def _run(exe, *args):
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, timeout=240, env=ENV)
    assert r.returncode == 0 and "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stdout + r.stderr
    return r.stdout


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_oracle_under_sanitizers(tmp_path, san):
    exe = _build(tmp_path, "gcc", "-std=c11", ["-fsanitize=" + san], ORACLE_SOURCES,
                 [os.path.join(ROOT, "oracle")], "san_oracle")
    assert "oracle ok" in _run(exe, 20011 if san == "thread" else 100003, 4)


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_host_code_under_sanitizers(tmp_path, san):
    exe = _build(tmp_path, "g++", "-std=c++17", ["-fsanitize=" + san], HOST_SOURCES,
                 [os.path.join(ROOT, "include"), CSRC], "san_host")
    out = _run(exe, 20000, 5000, 300) if san != "thread" else _run(exe, 200, 200, 300)
    assert "pool:" in out
