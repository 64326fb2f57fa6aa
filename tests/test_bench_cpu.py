"""Host logic of bench.py that needs no GPU: argument checks, the exact
integer closed forms it validates against, and the metric records."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_closed_forms_are_the_integer_recurrences():
    # listing order: a = 15^k, b = 3*15^(k-1), c = 4*15^(k-1)
    for k in range(1, 14):
        assert bench.expected_integers("listing", k) == (15.0 ** k, 3.0 * 15 ** (k - 1), 4.0 * 15 ** (k - 1))
    assert bench.expected_integers("copy_b", 10) == (1015254.0, 211896.0, 267786.0)
    with pytest.raises(AssertionError):  # beyond 2^53 the integers are not exact
        bench.expected_integers("listing", 14)


@pytest.mark.parametrize("args,code,text", [(["--gpus", "2"], 2, "exactly one GPU"),
                                            (["--legs", "nope"], 1, "unknown legs"),
                                            (["--steps", "0"], 1, "--steps")])
def test_argument_checks_before_any_gpu_work(args, code, text):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == code and text in r.stderr, (r.returncode, r.stderr)


def test_metric_records():
    kernel = {"cfg": {"block": 256}, "best_ms": 0.3, "avg_ms": 0.31, "best_GBps": 6500.0, "avg_GBps": 6400.0,
              "pct_peak_avg": 80.0}
    result = {"config": {"n": 1 << 27}, "roofline": {"traffic": 3.22e9},
              "per_kernel": {op: dict(kernel) for op in ("copy", "scale", "add", "triad")},
              "sweep": {"f64_aligned": {"2^16": {"regime": "L2", "copy_GBps": 400.0, "triad_GBps": 600.0}},
                        "f32_offset1_plus7": {"2^20": {"regime": "L2", "copy_GBps": 5000.0}}},
              "reduced_precision": {"bf16": {"triad": {"GBps": 6300.0, "max_rel_err_vs_f64": 3.8e-3}}},
              "batched": {"triad_best_GBps": 6400.0, "triad_avg_GBps": 6390.0, "total_elems": 10, "cfg": {},
                          "instances": 2}}
    recs = bench.metric_records(result)
    by = {}
    for r in recs:
        by.setdefault(r["config"], []).append(r)
    assert len(by["C2"]) == 4 and [r["traffic_bytes"] for r in by["C2"]].count(3.22e9) == 1
    assert len(by["C3"]) == 3
    assert {(r["dtype"], r["n"], r["offset"]) for r in by["C3"]} == {("f64", 1 << 16, 0), ("f32", (1 << 20) + 7, 1)}
    assert by["C4"][0]["rel_err_max"] == 3.8e-3 and by["C5"][0]["instances"] == 2


def test_profiler_runs_follow_the_rules():
    """Each rocprofv3 run names the program directly after `--`; counter runs
    collect one counter each and combine it with no trace option."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("_prof", os.path.join(ROOT, "paper_2206_06302_amd", "profiling.py"))
    prof = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(prof)
    assert prof.source_digest() == bench.kernel_source_digest()
    names = []
    for name, cmd, out in prof.runs("/tmp/raw"):
        names.append(name)
        assert cmd[0] == "rocprofv3"
        after = cmd[cmd.index("--") + 1:]
        assert after[0] == sys.executable and after[1].endswith("bench.py")
        if "--pmc" in cmd:
            assert len(cmd[cmd.index("--pmc") + 1].split()) == 1
            assert not {"--kernel-trace", "--sys-trace", "--runtime-trace", "-s", "-r"} & set(cmd[:cmd.index("--")])
    assert names == ["headline trace", "batched trace", "fetch counters", "write counters"]
