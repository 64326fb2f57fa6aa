"""Host logic of bench.py that needs no GPU: argument checks, the exact
integer closed forms it validates against, and the metric records."""
import os
import struct
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def test_exact_chain_closed_forms():
    # listing order: a = 15^k, b = 3*15^(k-1), c = 4*15^(k-1), exact below 2^53
    for k in range(1, 14):
        assert bench.exact_chain(1.0, 2.0, 0.0, 3.0, k) == (15.0 ** k, 3.0 * 15 ** (k - 1), 4.0 * 15 ** (k - 1))
    assert bench.exact_chain(1.0, 2.0, 0.0, 3.0, 10, "copy_b") == (1015254.0, 211896.0, 267786.0)
    assert bench.exact_chain(1.0, 2.0, 0.0, 3.0, 21, "copy_b") == (2361723449706.0, 492920384850.0, 622934354952.0)


def test_exact_chain_tells_a_fused_triad_from_an_unfused_one():
    """The 50-iteration check of the benchmark: the chain's bits with one
    rounding in the triad, and the unfused chain differs in a."""
    a, b, c = bench.exact_chain(1.0, 2.0, 0.0, 3.0, 50)
    assert (_bits(a), _bits(b), _bits(c)) == (0x4C2450D7D0D568D7, 0x4C0040ACA71120AC, 0x4C05AB90DEC180E5)
    au, bu, cu = bench.exact_chain(1.0, 2.0, 0.0, 3.0, 50, fused=False)
    assert (_bits(au), _bits(bu), _bits(cu)) == (0x4C2450D7D0D568D6, 0x4C0040ACA71120AB, 0x4C05AB90DEC180E4)
    # at 21 iterations (one warm-up plus 20 timed) both agree: 21 alone could not tell
    assert bench.exact_chain(1.0, 2.0, 0.0, 3.0, 21) == bench.exact_chain(1.0, 2.0, 0.0, 3.0, 21, fused=False)


def test_exact_chain_equals_the_oracle(oracle_lib):
    """Per-instance q of the batched workload and K up to 80: the helper
    reproduces the oracle's chain (std fma) bit for bit; past binary64's range
    every value is infinite."""
    import numpy as np

    import tsgen
    qs = list(tsgen.batched_scalars(5, 64)) + [3.0, 0.5, 4.0]
    for q in qs:
        for k in (1, 7, 21, 50, 80):
            assert bench.exact_chain(1.0, 2.0, 0.0, float(q), k) == oracle_lib.stream_scalar_f64(1.0, 2.0, 0.0, float(q), k)
    assert bench.exact_chain(1.0, 2.0, 0.0, 3.0, 300) == (float("inf"),) * 3
    assert oracle_lib.stream_scalar_f64(1.0, 2.0, 0.0, 3.0, 300) == (float("inf"),) * 3
    rng = np.random.default_rng(7)
    x = rng.standard_normal(4000) * np.exp2(rng.integers(-60, 60, 4000))
    y = rng.standard_normal(4000) * np.exp2(rng.integers(-60, 60, 4000))
    d = np.zeros_like(x)
    oracle_lib.op(oracle_lib.F64, oracle_lib.TRIAD, x, y, d, 3.0)
    assert all(bench._fma(3.0, float(yv), float(xv)) == dv for xv, yv, dv in zip(x, y, d))


def test_summary_is_the_last_key():
    kernel = {"best_GBps": 6500.0, "avg_GBps": 6400.0, "pct_peak_best": 81.25, "pct_peak_avg": 80.0, "bytes": 1,
              "best_ms": 1.0, "avg_ms": 1.0, "cfg": {}}
    result = {"metric": "m", "value": 1.0, "per_kernel": {op: dict(kernel) for op in bench.OPS},
              "roofline": {"frac": 0.8}, "valid": {"timed_arrays": True, "k50_fused_chain": True},
              "ceiling": {name: {"avg_GBps": 6600.0} for name, _, _ in bench.PROBE_KINDS},
              "batched": {"triad_best_GBps": 6300.0, "triad_avg_GBps": 6290.0, "triad_vs_plain_n2p27_triad": 0.97,
                          "graph_iteration_GBps": 6200.0, "valid_after_graph_replays": True,
                          "valid_after_map_launches": True,
                          "maps": {op: {"avg_GBps": 6208.0} for op in bench.OPS},
                          "maps_avg_vs_plain_avg": {op: 0.97 for op in bench.OPS}},
              "cpu_baseline": {"value": 250.0, "cores": 16, "valid": True}, "sweep": {}}
    out = bench.order_for_output(result)
    keys = list(out)
    assert keys[-4:] == ["per_kernel", "roofline", "cpu_baseline", "summary"] and keys[:2] == ["metric", "value"]
    s = out["summary"]
    assert s["triad_avg_vs_2r1w_ceiling"] == round(6400 / 6600, 4) and s["batched"]["valid"] is True
    assert "triad 6500/6400" in bench.summary_text(s)
    assert s["batched"]["maps_avg_GBps"]["copy"] == 6208.0 and "copy 6208 (0.970)" in bench.summary_text(s)


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
            counters = cmd[cmd.index("--pmc") + 1:cmd.index("--output-format")]
            # within one pass: at most 4 TCC counters (FETCH_SIZE alone takes 3, WRITE_SIZE 2)
            tcc = sum(3 if c == "FETCH_SIZE" else 2 if c == "WRITE_SIZE" else int(c.startswith("TCC_"))
                      for c in counters)
            assert 1 <= len(counters) and tcc <= 4, counters
            assert not {"--kernel-trace", "--sys-trace", "--runtime-trace", "-s", "-r"} & set(cmd[:cmd.index("--")])
    assert names == ["headline trace", "batched trace", "reduced trace", "fetch counters", "write counters",
                     "read requests", "write requests"]
