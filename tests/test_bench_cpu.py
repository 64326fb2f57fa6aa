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
    assert names == ["headline trace", "batched trace", "reduced trace", "validation trace", "fetch counters",
                     "write counters", "read requests", "write requests"]


def _load_profiling():
    import importlib.util

    spec = importlib.util.spec_from_file_location("_prof", os.path.join(ROOT, "paper_2206_06302_amd", "profiling.py"))
    prof = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(prof)
    return prof


def _write_csv(path, header, rows):
    import csv

    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def _synthetic_raw(raw):
    """A raw profiler directory whose figures have answers known by
    construction: 2^30-byte arrays, read requests of 128 bytes (plus, for
    copy, four of 32 bytes standing in for one 128-byte one), write requests
    of 64 bytes, and a small-grid launch of every map that the summaries must
    leave out."""
    import json

    gib = 1 << 30
    plain = "void ts::stream_kernel<0, {op}, 16, 1, true, true>(void const*, void const*, void*, double, float)"
    batch = "void ts::batch_kernel<0, {op}, 1, 1, true, true, true>(ts::BatchTile const*, unsigned long)"
    probe = {"read_1r": "void ts::probe_kernel<16, 1, 0, 1, true, true, false>(void const*)",
             "write_1w": "void ts::probe_kernel<16, 0, 1, 1, true, true, false>(void const*)",
             "copy_1r1w": "void ts::probe_kernel<16, 1, 1, 1, true, true, false>(void const*)"}
    big, small = 1 << 24, 1 << 10

    def req(reads, writes, copy=False):
        rd32 = 4 if copy else 0
        rd = reads // 128 - (1 if copy else 0) + rd32
        wr = writes // 64
        return {"FETCH_SIZE": rd * 64 / 1024, "WRITE_SIZE": wr * 64 / 1024, "TCC_EA0_RDREQ_sum": rd,
                "TCC_EA0_RDREQ_32B_sum": rd32, "TCC_BUBBLE_sum": 0, "TCC_EA0_RDREQ_DRAM_sum": rd,
                "TCC_EA0_WRREQ_sum": wr, "TCC_EA0_WRREQ_64B_sum": wr, "TCC_EA0_WRREQ_DRAM_sum": wr}

    launches = []  # (kernel name, grid, counters) per dispatch
    for op, arrays in ((0, 2), (1, 2), (2, 3), (3, 3)):
        launches += [(plain.format(op=op), big, req((arrays - 1) * gib, gib, copy=op == 0))] * 2
        launches.append((plain.format(op=op), small, req(4096, 4096)))
        launches.append((batch.format(op=op), big, req((arrays - 1) * 3 * gib, 3 * gib)))
    launches += [(probe["read_1r"], big, req(gib, 0)), (probe["write_1w"], big, req(0, gib)),
                 (probe["copy_1r1w"], big, req(gib, gib))]
    prof = _load_profiling()
    header = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    for _, sub, counters in prof.PMC_RUNS:
        rows = [[i, g, name, c, vals[c]] for i, (name, g, vals) in enumerate(launches) for c in counters]
        _write_csv(os.path.join(raw, sub, "run_counter_collection.csv"), header, rows)
        with open(os.path.join(raw, sub + ".json"), "w") as f:
            f.write(json.dumps({"batched": {"total_elems": 3 * (1 << 27), "tiles": 12345}}) + "\n")

    stats = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
    # 2 or 3 GiB of STREAM bytes in 400 or 600 µs: 5368.7 GB/s avg; minimum 1.25x faster
    rows = [[plain.format(op=op), 71, 0, 200e3 * a, 0, 160e3 * a, 250e3 * a, 0]
            for op, a in ((0, 2), (1, 2), (2, 3), (3, 3))]
    rows.append(["void ts::(anonymous namespace)::fill_const_kernel<0>(void*, unsigned long)", 3, 0, 1e5, 0, 1e5,
                 1e5, 0])
    _write_csv(os.path.join(raw, "trace_headline", "run_kernel_stats.csv"), stats, rows)
    per = {op: {"avg_ms": 0.5, "avg_GBps": 1.0, "best_ms": 0.4} for op in ("copy", "scale", "add", "triad")}
    with open(os.path.join(raw, "trace_headline.json"), "w") as f:
        f.write("log line\n" + json.dumps({"per_kernel": per}) + "\n")

    rows = [[batch.format(op=op), 11, 0, 3 * 200e3 * a, 0, 3 * 160e3 * a, 3 * 250e3 * a, 0]
            for op, a in ((0, 2), (1, 2), (2, 3), (3, 3))]
    _write_csv(os.path.join(raw, "trace_batched", "run_kernel_stats.csv"), stats, rows)
    bb = {"total_elems": 3 * (1 << 27), "tiles": 12345, "tile_elems": 1024,
          "cfg": {"block": 1024, "unroll": 1, "tiles_per_wg": 1, "grid_per_cu": 0, "nt_load": 1, "nt_store": 1,
                  "record_ahead": 1},
          "graph_iteration_ms": 5.0, "graph_iteration_GBps": 5000.0, "triad_best_GBps": 6000.0,
          "triad_avg_GBps": 5900.0, "plain_per_instance_triad_best_GBps": 4000.0,
          "maps": {op: {"avg_GBps": 5800.0} for op in ("copy", "scale", "add", "triad")},
          "valid_after_graph_replays": True}
    with open(os.path.join(raw, "trace_batched.json"), "w") as f:
        f.write(json.dumps({"batched": bb}) + "\n")

    trace = ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for dt, nbytes in ((0, 8), (1, 4), (2, 2)):
        name = f"void ts::stream_kernel<{dt}, 3, 16, 1, true, true>(void const*, void const*, void*)"
        # 2^28 elements: 3 * 2^28 * nbytes bytes in (nbytes / 8) ms; a small launch that must be left out
        rows += [[name, 1 << 22, 0, int(nbytes / 8 * 1e6)]] * 2 + [[name, 1 << 10, 0, 1]]
    _write_csv(os.path.join(raw, "trace_reduced", "run_kernel_trace.csv"), trace, rows)
    with open(os.path.join(raw, "trace_reduced.json"), "w") as f:
        f.write(json.dumps({"reduced_precision": {"f32": {"triad": {"GBps": 1.5}}}}) + "\n")

    trace = ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size"]
    cs = "void ts::(anonymous namespace)::checksum_pass1<{dt}, 0>(void const*, unsigned long, double, ts::CsPart*, unsigned int)"
    fill = "void ts::(anonymous namespace)::fill_const_kernel<{dt}>(void*, unsigned long, double, unsigned long, unsigned long)"
    uni = "void ts::(anonymous namespace)::fill_uniform_kernel<{dt}>(void*, unsigned long, unsigned long, unsigned long, double, double, unsigned long, unsigned long)"
    mm = "void ts::(anonymous namespace)::mismatch_pass1<{dt}>(void const*, void const*, unsigned long, ts::CsPart*, unsigned int)"
    rows = []
    for dt in range(4):
        # 2^30 bytes in 100 µs (checksum) and 200 µs (fill); small launches that must be left out
        rows += [[cs.format(dt=dt), 4096 * 256, 0, 100000, 65536]] * 3 + [[cs.format(dt=dt), 256, 0, 1, 65536]]
        rows += [[fill.format(dt=dt), 262144 * 256, 0, 200000, 0]] * 2 + [[fill.format(dt=dt), 256, 0, 1, 0]]
        rows += [[uni.format(dt=dt), 262144 * 256, 0, 250000, 0]] * 2
        # two arrays of 2^30 bytes read in 400 µs
        rows += [[mm.format(dt=dt), 8192 * 256, 0, 400000, 0]] + [[mm.format(dt=dt), 256, 0, 1, 0]]
    rows += [["void ts::(anonymous namespace)::reduce_pass2(ts::CsPart const*, unsigned int, ts::CsPart*)", 256, 0,
              5000, 8192]] * 4
    _write_csv(os.path.join(raw, "trace_validation", "run_kernel_trace.csv"), trace, rows)
    with open(os.path.join(raw, "trace_validation.json"), "w") as f:
        f.write(json.dumps({"validation": {"bf16": {"checksum_call_avg_GBps": 2.5, "fill_const_avg_GBps": 3.5,
                                                    "mismatch_call_avg_GBps": 4.5}}}) + "\n")
    return prof


def test_profile_summaries_from_known_counts(tmp_path, monkeypatch):
    """The summaries turn request counts into bytes, keep the 2^27 launches
    apart from smaller ones of the same kernel, and leave the triad's bytes
    and the kernel digest where bench.py reads them."""
    raw, out = str(tmp_path / "raw"), str(tmp_path / "profiles")
    prof = _synthetic_raw(raw)
    prof.summarize(raw, out)
    assert sorted(os.listdir(out)) == ["batched_f64_4096_kernel_trace.md", "batched_f64_4096_pmc.md",
                                       "checksum_fill_1gib_kernel_trace.md",
                                       "stream_f64_n2p27_kernel_trace.md", "stream_f64_n2p27_pmc.md",
                                       "stream_reduced_n2p28_kernel_trace.md"]
    read = lambda f: open(os.path.join(out, f)).read()  # noqa: E731

    pmc = read("stream_f64_n2p27_pmc.md")
    rows = {ln.split("|")[1].strip(): ln for ln in pmc.splitlines() if ln.startswith("| ")}
    for op in ("copy", "scale", "add", "triad"):
        assert rows[op].rstrip().endswith("| 1.0000 |"), rows[op]
        assert rows[op].split("|")[2].strip() == "2/2/2/2"  # the small-grid launch is left out
    # the probe's read requests carry 128 bytes each, its write requests 64
    assert "| 128.00 | – |" in rows["read_1r"] and "| – | 64.00 |" in rows["write_1w"]
    assert "traffic_bytes_per_launch: 3.221225e+09" in pmc
    assert f"kernel_source_digest: {prof.source_digest()}" in pmc
    assert "$RAW/pmc_fetch" in pmc and raw not in pmc

    bpmc = read("batched_f64_4096_pmc.md")
    assert "traffic_bytes_per_launch (triad): 9.663676e+09" in bpmc
    assert all(r.rstrip().endswith("| 1.0000 |") for r in bpmc.splitlines() if r.startswith("| triad |"))

    trace = read("stream_f64_n2p27_kernel_trace.md")
    lines = [ln for ln in trace.splitlines() if ln.startswith("| `stream_kernel<f64,")]
    assert len(lines) == 4 and all("| 5368.7 | 6710.9 |" in ln for ln in lines), lines
    assert "| `fill_const_kernel<0>` | – | 3 |" in trace

    btrace = read("batched_f64_4096_kernel_trace.md")
    lines = [ln for ln in btrace.splitlines() if ln.startswith("| `batch_kernel<f64,")]
    assert len(lines) == 4 and all("record_ahead=1>`" in ln and "| 5368.7 | 6710.9 |" in ln for ln in lines)

    red = read("stream_reduced_n2p28_kernel_trace.md")
    rows = {ln.split("|")[1].strip(): ln.split("|") for ln in red.splitlines()
            if ln.split("|")[1:2] and ln.split("|")[1].strip() in ("f64", "f32", "bf16", "f16")}
    assert rows["f64"][4].strip() == "2" and rows["f64"][6].strip() == "6442.5"
    # elements per second against binary64: 2x for 4-byte storage, 4x for 2-byte storage
    assert rows["f32"][8].strip() == "2.00" and rows["bf16"][8].strip() == "4.00"
    assert rows["f32"][9].strip() == "1.5"

    val = read("checksum_fill_1gib_kernel_trace.md")
    rows = [ln.split("|") for ln in val.splitlines() if ln.startswith("| ") and "`" in ln]
    assert len(rows) == 16
    for r in rows:  # the small-grid launches are left out
        if "checksum_pass1" in r[2]:
            assert [c.strip() for c in r[3:7]] == ["4096", "3", "100.0", "10737.4"], r
        elif "fill_const" in r[2]:
            assert [c.strip() for c in r[3:7]] == ["262144", "2", "200.0", "5368.7"], r
        elif "fill_uniform" in r[2]:
            assert [c.strip() for c in r[3:7]] == ["262144", "2", "250.0", "4295.0"], r
        else:
            assert [c.strip() for c in r[3:7]] == ["8192", "1", "400.0", "5368.7"], r
    bf16 = [r for r in rows if r[1].strip() == "bf16"]
    assert [r[7].strip() for r in bf16] == ["2.5", "3.5", "", "4.5"]
    assert "averages 5.0 µs over 4 dispatches" in val
    assert "--legs validation" in val

    monkeypatch.setattr(bench, "PROFILE_PMC", os.path.join(out, "stream_f64_n2p27_pmc.md"))
    assert bench.committed_traffic() == 3.221225e9
    with open(bench.PROFILE_PMC, "w") as f:
        f.write(pmc.replace(prof.source_digest(), "0" * 16))
    assert bench.committed_traffic() is None
