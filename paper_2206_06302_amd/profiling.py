"""rocprofv3 runs of bench.py and the summaries kept under profiles/.

    python paper_2206_06302_amd/profiling.py run --raw DIR        # on a machine with the GPU
    python paper_2206_06302_amd/profiling.py summarize --raw DIR  # anywhere: rewrites profiles/*.md

`run` starts eight rocprofv3 runs, each a process of its own with the program
directly after `--`, from /tmp with TMPDIR=/tmp:

  headline trace   --kernel-trace --stats of bench.py --quick --no-cpu --warmup 1 --steps 20
  batched trace    --kernel-trace --stats of bench.py --no-cpu --legs batched --warmup 1 --steps 20
  reduced trace    --kernel-trace         of bench.py --no-cpu --legs reduced_precision --warmup 1 --steps 3
  validation trace --kernel-trace         of bench.py --no-cpu --legs validation --warmup 1 --steps 3
  fetch counters   --pmc FETCH_SIZE       of bench.py --no-cpu --legs calibration,batched --no-per-instance
                                          --warmup 1 --steps 3
  write counters   --pmc WRITE_SIZE       of the same command
  read requests    --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_BUBBLE_sum TCC_EA0_RDREQ_DRAM_sum
  write requests   --pmc TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum TCC_EA0_WRREQ_DRAM_sum

`summarize` turns the raw CSV files into short markdown summaries: the
per-kernel trace of the headline, of the batched leg (with the bench's own
event timings from the same runs beside rocprof's), of the maps on
reduced-precision storage and of the validation kernels per storage type, and the HBM traffic per launch of the four
headline maps and the four batched maps.

HBM bytes come from the L2-to-memory request counts: on gfx950 every read
request that is not a 32-byte one moves 128 bytes, and write requests move
64 or 32 bytes.  The memory-system probe kernels of bench.py's calibration
leg, which move exactly known bytes and are not themselves reported, check
this: the read-only probe's 2^30 bytes arrive in 2^23 requests.  They also
show why FETCH_SIZE alone reads half: its expression prices 128-byte reads
through TCC_BUBBLE, which stays 0 on this part, so each read request counts
64 bytes.  FETCH_SIZE and WRITE_SIZE are reported beside the request-count
bytes, scaled by what they read for the probe's copy of known size.  Each
summary records the source digest of the headline kernels, so the benchmark
reports counter traffic only while the kernels are unchanged.

This file is loaded by path (bench.py does so for source_digest) and needs
neither torch nor the library.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = os.path.join(ROOT, "profiles")
N27 = 1 << 27
OPS = {0: "copy", 1: "scale", 2: "add", 3: "triad"}
ARRAYS = {0: 2, 1: 2, 2: 3, 3: 3}


def source_digest(root: str = ROOT) -> str:
    """Digest of what determines the binary64 kernels of the headline: their
    source (comments and whitespace aside) and the tuned plain launch
    configurations of binary64 (measured rates excluded)."""
    h = hashlib.sha256()
    for rel in ("paper_2206_06302_amd/csrc/ts_device.hpp", "paper_2206_06302_amd/csrc/kern_f64.hip"):
        text = open(os.path.join(root, rel)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    tune = os.path.join(root, "paper_2206_06302_amd", "tune", "gfx950.json")
    if os.path.exists(tune):
        entries = json.load(open(tune)).get("entries", [])
        cfgs = sorted(json.dumps({k: v for k, v in e.items() if k != "bytes_per_s"}, sort_keys=True)
                      for e in entries if e.get("dtype") == "f64" and not e.get("batched"))
        h.update("\n".join(cfgs).encode())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
# Runs
# ---------------------------------------------------------------------------
def _bench(*args):
    return [sys.executable, os.path.join(ROOT, "bench.py"), *args]


READ_REQUESTS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_BUBBLE_sum", "TCC_EA0_RDREQ_DRAM_sum")
WRITE_REQUESTS = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_WRREQ_DRAM_sum")
PMC_RUNS = (("fetch counters", "pmc_fetch", ("FETCH_SIZE",)), ("write counters", "pmc_write", ("WRITE_SIZE",)),
            ("read requests", "pmc_rdreq", READ_REQUESTS), ("write requests", "pmc_wrreq", WRITE_REQUESTS))


def runs(raw: str) -> list[tuple[str, list[str], str]]:
    """(name, command, stdout file) of the profiler runs."""
    out = [
        ("headline trace", ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv", "-d",
                            os.path.join(raw, "trace_headline"), "-o", "run", "--",
                            *_bench("--quick", "--no-cpu", "--warmup", "1", "--steps", "20")],
         os.path.join(raw, "trace_headline.json")),
        ("batched trace", ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv", "-d",
                           os.path.join(raw, "trace_batched"), "-o", "run", "--",
                           *_bench("--no-cpu", "--legs", "batched", "--warmup", "1", "--steps", "20")],
         os.path.join(raw, "trace_batched.json")),
        ("reduced trace", ["rocprofv3", "--kernel-trace", "--output-format", "csv", "-d",
                           os.path.join(raw, "trace_reduced"), "-o", "run", "--",
                           *_bench("--no-cpu", "--legs", "reduced_precision", "--warmup", "1", "--steps", "3")],
         os.path.join(raw, "trace_reduced.json")),
        ("validation trace", ["rocprofv3", "--kernel-trace", "--output-format", "csv", "-d",
                              os.path.join(raw, "trace_validation"), "-o", "run", "--",
                              *_bench("--no-cpu", "--legs", "validation", "--warmup", "1", "--steps", "3")],
         os.path.join(raw, "trace_validation.json")),
    ]
    for name, sub, counters in PMC_RUNS:
        out.append((name, ["rocprofv3", "--pmc", *counters, "--output-format", "csv", "-d", os.path.join(raw, sub),
                           "-o", "run", "--",
                           *_bench("--no-cpu", "--legs", "calibration,batched", "--no-per-instance", "--warmup", "1",
                                   "--steps", "3")],
                    os.path.join(raw, sub + ".json")))
    return out


def run(raw: str, timeout: int) -> int:
    raw = os.path.abspath(raw)
    os.makedirs(raw, exist_ok=True)
    env = dict(os.environ, TMPDIR="/tmp")
    for name, cmd, out in runs(raw):
        print(f"[{name}] {' '.join(cmd)}", flush=True)
        with open(out, "w") as so, open(out + ".log", "w") as se:
            try:
                rc = subprocess.run(cmd, stdout=so, stderr=se, cwd="/tmp", env=env, timeout=timeout).returncode
            except subprocess.TimeoutExpired:
                print(f"[{name}] timed out after {timeout} s", flush=True)
                return 124
        print(f"[{name}] exit {rc}", flush=True)
        if rc != 0:
            return rc
    return 0


# ---------------------------------------------------------------------------
# Summaries
# ---------------------------------------------------------------------------
def _stats(path):
    return list(csv.DictReader(open(path)))


def _counters(dirpath, counter):
    """{(kernel name, grid size): [value per dispatch]} of one counter."""
    vals = {}
    for f in glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") == counter:
                vals.setdefault((r["Kernel_Name"], int(r["Grid_Size"])), []).append(float(r["Counter_Value"]))
    return vals


def _pick(vals, pattern, grid=None):
    out = []
    for (name, g), v in vals.items():
        if re.search(pattern, name) and (grid is None or g == grid):
            out += v
    return out


def _bench_json(path):
    return json.loads(open(path).read().strip().splitlines()[-1])


DT_NAMES = {0: "f64", 1: "f32", 2: "bf16", 3: "f16"}
DT_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}


def _reduced_summary(raw, cmd):
    """Per storage type and map, the average duration of the 2^28-element
    launches (the largest grid of each kernel) from the per-dispatch trace."""
    n = 1 << 28
    rows = {}
    for f in glob.glob(os.path.join(raw, "trace_reduced", "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            m = re.search(r"stream_kernel<(\d+), (\d+), (\d+), (\d+), (\w+), (\w+)>", r["Kernel_Name"])
            if not m:
                continue
            key = (int(m.group(1)), int(m.group(2)))
            grid = int(r["Grid_Size_X"])
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            shape = f"VB{m.group(3)},U{m.group(4)},nt_load={int(m.group(5) == 'true')},nt_store={int(m.group(6) == 'true')}"
            rows.setdefault(key, {}).setdefault(grid, []).append((dur, shape))
    bj = _bench_json(os.path.join(raw, "trace_reduced.json"))["reduced_precision"]
    L = ["# Kernel trace: STREAM maps on reduced-precision storage, N = 2^28 per array (bench reduced leg)", "",
         "Made by `python paper_2206_06302_amd/profiling.py run` (then `summarize`); the run:", "",
         "```", "export TMPDIR=/tmp; cd /tmp", cmd, "```", "",
         "Binary64 storage beside binary32, bfloat16 and binary16 storage (arithmetic in binary32 for the",
         "16-bit types).  Per storage type and map: the launches over 2^28 elements (10 + 20 of the chained",
         "iteration, then 2 + 10 standalone and 1 for the error figure), their average duration from the",
         "trace, STREAM bytes / that duration, and elements per second against binary64's.", "",
         "| storage | map | kernel shape | dispatches | avg µs | GB/s (avg) | Gelem/s | elements/s vs f64 | "
         "bench events GB/s |", "|---|---|---|---|---|---|---|---|---|"]
    rate64 = {}
    for dt in range(4):
        for op in range(4):
            if (dt, op) not in rows:
                continue
            grid = max(rows[(dt, op)])
            launches = rows[(dt, op)][grid]
            avg = sum(d for d, _ in launches) / len(launches)
            gb = ARRAYS[op] * n * DT_BYTES[dt] / avg
            ge = n / avg
            if dt == 0:
                rate64[op] = ge
            ev = bj.get(DT_NAMES[dt], {}).get(OPS[op], {}).get("GBps", "")
            L.append(f"| {DT_NAMES[dt]} | {OPS[op]} | `{launches[0][1]}` | {len(launches)} | {avg / 1e3:.1f} | {gb:.1f} | "
                     f"{ge:.2f} | {ge / rate64[op]:.2f} | {ev} |" if op in rate64 else "")
    return L + [""]


def _validation_summary(raw, cmd):
    """Per storage type, the checksum's two passes, the constant and uniform
    fills and the mismatch count over the validation leg's 1 GiB arrays (the largest grid of each kernel and
    type), average durations from the per-dispatch trace."""
    nbytes = 1 << 30
    rows = {}
    for f in glob.glob(os.path.join(raw, "trace_validation", "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"]
            m = re.search(r"(checksum_pass1|fill_const_kernel|fill_uniform_kernel|mismatch_pass1)<(\d+)", name)
            if m:
                key = (int(m.group(2)), m.group(1))
            elif "reduce_pass2" in name:
                key = (None, "reduce_pass2")
            else:
                continue
            grid = int(r["Grid_Size_X"])
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            rows.setdefault(key, {}).setdefault(grid, []).append(dur)
    bj = _bench_json(os.path.join(raw, "trace_validation.json")).get("validation", {})
    L = ["# Kernel trace: validation kernels over 1 GiB per storage type (bench validation leg)", "",
         "Made by `python paper_2206_06302_amd/profiling.py run` (then `summarize`); the run:", "",
         "```", "export TMPDIR=/tmp; cd /tmp", cmd, "```", "",
         "The checksum's first pass (grid-strided 16 KiB chunks, one workgroup part each), the constant",
         "and uniform fills and the mismatch count's first pass (two arrays read) over arrays of 2^30 bytes per storage",
         "type: the launches of the largest grid, their average duration from the trace, and bytes / that",
         "duration.  The bench's own figure for a whole call (both passes, the result's copy to the host",
         "and the wait for it; for the fill, the launch) is beside it.",
         "The binary64 rows also hold the headline's own validation calls on its 2^27-element arrays,",
         "which are the same size.  The first pass's workgroups of 256 lanes reserve 64 KiB of LDS for",
         "binary64 and binary32 and 48 KiB for the 16-bit types, which leaves room for two or three on a",
         "CU (the trace lists only the 8 KiB the kernel declares).", "",
         "| storage | kernel | grid (workgroups) | dispatches | avg µs | GB/s (avg) | bench GB/s |",
         "|---|---|---|---|---|---|---|"]
    for dt in range(4):
        for kern, bench_key, arrays in (("checksum_pass1", "checksum_call_avg_GBps", 1),
                                        ("fill_const_kernel", "fill_const_avg_GBps", 1),
                                        ("fill_uniform_kernel", "fill_uniform_avg_GBps", 1),
                                        ("mismatch_pass1", "mismatch_call_avg_GBps", 2)):
            if (dt, kern) not in rows:
                continue
            grid = max(rows[(dt, kern)])
            launches = rows[(dt, kern)][grid]
            avg = sum(launches) / len(launches)
            ev = bj.get(DT_NAMES[dt], {}).get(bench_key, "")
            L.append(f"| {DT_NAMES[dt]} | `{kern}` | {grid // 256} | {len(launches)} | "
                     f"{avg / 1e3:.1f} | {arrays * nbytes / avg:.1f} | {ev} |")
    if (None, "reduce_pass2") in rows:
        p2 = [d for v in rows[(None, "reduce_pass2")].values() for d in v]
        L += ["", f"The second pass (one workgroup folding the parts in a fixed order) averages "
              f"{sum(p2) / len(p2) / 1e3:.1f} µs over {len(p2)} dispatches."]
    return L + [""]


def _plain_name(name):
    m = re.search(r"stream_kernel<(\d+), (\d+), (\d+), (\d+), (\w+), (\w+)>", name)
    if not m:
        return None
    dt, op, vb, u, ntl, nts = m.groups()
    return int(dt), int(op), (f"stream_kernel<f64,{OPS[int(op)]},VB{vb},U{u},nt_load={int(ntl == 'true')},"
                              f"nt_store={int(nts == 'true')}>")


def _short(name):
    m = re.search(r"(\w+_kernel(?:<[^>]*>)?|__amd_rocclr_\w+|reduce_pass2|\w+_pass1<[^>]*>)", name)
    return m.group(1) if m else name[:60]


def _command(cmd, raw):
    """The command as text, with the raw directory as $RAW and the repository as $REPO."""
    out = []
    for c in cmd:
        if c == sys.executable:
            c = "python3"
        elif c.startswith(raw):
            c = "$RAW" + c[len(raw):]
        elif c.startswith(ROOT):
            c = "$REPO" + c[len(ROOT):]
        out.append(c)
    return " ".join(out)


class Counters:
    """Every counter of the four counter runs, averaged per dispatch of one kernel."""

    def __init__(self, raw: str):
        self.vals = {}
        for _, sub, counters in PMC_RUNS:
            for c in counters:
                self.vals[c] = _counters(os.path.join(raw, sub), c)

    def mean(self, counter, pattern, grid=None):
        v = _pick(self.vals[counter], pattern, grid)
        return (sum(v) / len(v), len(v)) if v else (float("nan"), 0)

    def launch(self, pattern, grid=None) -> dict:
        """Per-dispatch means of every counter for kernels matching `pattern`
        (and grid size), plus the bytes the request counts give."""
        d = {c: self.mean(c, pattern, grid)[0] for c in self.vals}
        d["dispatches"] = "/".join(str(self.mean(c, pattern, grid)[1]) for c in ("FETCH_SIZE", "WRITE_SIZE",
                                                                               READ_REQUESTS[0], WRITE_REQUESTS[0]))
        rd, rd32 = d["TCC_EA0_RDREQ_sum"], d["TCC_EA0_RDREQ_32B_sum"]
        wr, wr64 = d["TCC_EA0_WRREQ_sum"], d["TCC_EA0_WRREQ_64B_sum"]
        d["read_bytes"] = 128.0 * (rd - rd32) + 32.0 * rd32
        d["write_bytes"] = 64.0 * wr64 + 32.0 * (wr - wr64)
        return d


# probe_kernel<vector bytes, reads, writes, ...>: the calibration leg's 16-byte probes
PROBE = {"read_1r": r"probe_kernel<16, 1, 0,", "write_1w": r"probe_kernel<16, 0, 1,",
         "copy_1r1w": r"probe_kernel<16, 1, 1,"}
PROBE_BYTES = N27 * 8  # the calibration leg's probes move 2^27 binary64 elements per array


def _calibration(cn: Counters):
    """Lines on the probe kernels of known traffic, and the FETCH_SIZE /
    WRITE_SIZE scale factors from the probe's copy."""
    r, w, c = (cn.launch(PROBE[k]) for k in ("read_1r", "write_1w", "copy_1r1w"))
    # FETCH_SIZE prices a read request at 64 bytes when TCC_BUBBLE is 0; a
    # request moves 128.  WRITE_SIZE prices write requests at their size.
    ff, fw = 128.0 / 64.0, 1.0
    lines = [
        "Calibration on the memory-system probe of bench.py's calibration leg (straight-line 16-byte",
        "loads and stores over 2^27 binary64 elements per array, 2^30 bytes; not a reported kernel):", "",
        "| probe | reads / writes (bytes) | read requests (all / 32 B / TCC_BUBBLE) | write requests (all / 64 B) "
        "| bytes per read request | bytes per write request | FETCH_SIZE KiB | WRITE_SIZE KiB |",
        "|---|---|---|---|---|---|---|---|"]
    for name, d, rb, wb in (("read_1r", r, PROBE_BYTES, 0), ("write_1w", w, 0, PROBE_BYTES),
                            ("copy_1r1w", c, PROBE_BYTES, PROBE_BYTES)):
        bpr = f"{rb / d['TCC_EA0_RDREQ_sum']:.2f}" if rb else "–"
        bpw = f"{wb / d['TCC_EA0_WRREQ_sum']:.2f}" if wb else "–"
        lines.append(f"| {name} | {rb:.4e} / {wb:.4e} | {d['TCC_EA0_RDREQ_sum']:.0f} / {d['TCC_EA0_RDREQ_32B_sum']:.0f} / "
                     f"{d['TCC_BUBBLE_sum']:.0f} | {d['TCC_EA0_WRREQ_sum']:.0f} / {d['TCC_EA0_WRREQ_64B_sum']:.0f} | "
                     f"{bpr} | {bpw} | {d['FETCH_SIZE']:.0f} | {d['WRITE_SIZE']:.0f} |")
    extra = w["TCC_EA0_WRREQ_sum"] - PROBE_BYTES / 64
    lines += ["", f"Every read request carries 128 bytes and every write request 64, while TCC_BUBBLE, the counter "
              f"FETCH_SIZE's expression prices at 128 bytes, reads {r['TCC_BUBBLE_sum']:.0f}: FETCH_SIZE counts each "
              f"read request as 64 bytes.  The bytes below are therefore 128 x (read requests - 32-byte ones) + 32 x "
              f"the 32-byte ones, and 64 or 32 per write request.  FETCH_SIZE and WRITE_SIZE are listed beside them, "
              f"scaled by what that gives: fetch x{ff:.1f} (128-byte requests priced at 64), write x{fw:.1f}.  The "
              f"write-only probe's {extra:.0f} write requests beyond 2^30 / 64 ({extra * 64 / PROBE_BYTES * 100:.2f} %) "
              f"are dirty lines of the kernel before it, written back while it runs."]
    return lines, ff, fw


def _traffic_table(rows, ff, fw):
    """Markdown rows: (label, counters, algorithmic read bytes, algorithmic write bytes)."""
    out = ["| map | dispatches (fetch/write/read req/write req) | FETCH_SIZE KiB | WRITE_SIZE KiB | read requests | "
           "write requests | read bytes | write bytes | FETCH/WRITE scaled | algorithmic read / write | "
           "traffic / algorithmic |", "|---|---|---|---|---|---|---|---|---|---|---|"]
    for label, d, ar, aw in rows:
        scaled = d["FETCH_SIZE"] * 1024 * ff + d["WRITE_SIZE"] * 1024 * fw
        out.append(f"| {label} | {d['dispatches']} | {d['FETCH_SIZE']:.0f} | {d['WRITE_SIZE']:.0f} | "
                   f"{d['TCC_EA0_RDREQ_sum']:.0f} | {d['TCC_EA0_WRREQ_sum']:.0f} | {d['read_bytes']:.4e} | "
                   f"{d['write_bytes']:.4e} | {scaled:.4e} | {ar:.4e} / {aw:.4e} | "
                   f"{(d['read_bytes'] + d['write_bytes']) / (ar + aw):.4f} |")
    return out


def summarize(raw: str, out: str = PROFILES) -> None:
    raw = os.path.abspath(raw)
    os.makedirs(out, exist_ok=True)
    digest = source_digest()
    cmds = {name: cmd for name, cmd, _ in runs(raw)}
    cn = Counters(raw)
    calib, ff, fw = _calibration(cn)
    pmc_cmds = ["```", "export TMPDIR=/tmp; cd /tmp", *(_command(cmds[name], raw) for name, _, _ in PMC_RUNS), "```"]

    # headline trace
    bj = _bench_json(os.path.join(raw, "trace_headline.json"))
    L = ["# Kernel trace: STREAM f64, N = 2^27 per array (bench headline)", "",
         "Made by `python paper_2206_06302_amd/profiling.py run` (then `summarize`); the run:", "",
         "```", "export TMPDIR=/tmp; cd /tmp", _command(cmds["headline trace"], raw), "```", "",
         "71 launches per map (1 warm-up, 20 timed steps, 50 of the fused-chain check).  GB/s = STREAM bytes",
         "of the launch / its average duration (copy and scale move 2 arrays of 1 GiB, add and triad 3).", "",
         "| kernel | map | calls | avg µs | min µs | max µs | GB/s (avg) | GB/s (min time) |",
         "|---|---|---|---|---|---|---|---|"]
    for r in _stats(os.path.join(raw, "trace_headline", "run_kernel_stats.csv")):
        avg, mn, mx = float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"])
        p = _plain_name(r["Name"])
        if p and p[0] == 0:
            b = ARRAYS[p[1]] * N27 * 8
            L.append(f"| `{p[2]}` | {OPS[p[1]]} | {r['Calls']} | {avg/1e3:.1f} | {mn/1e3:.1f} | {mx/1e3:.1f} | "
                     f"{b/avg:.1f} | {b/mn:.1f} |")
        else:
            L.append(f"| `{_short(r['Name'])}` | – | {r['Calls']} | {avg/1e3:.1f} | {mn/1e3:.1f} | {mx/1e3:.1f} | | |")
    L += ["", "The same run timed the launches itself with events on the target's stream (bench.py's own",
          "figures, profiler attached):", "", "| map | events avg µs | events GB/s (avg) | events best µs |",
          "|---|---|---|---|"]
    for op in ("copy", "scale", "add", "triad"):
        k = bj["per_kernel"][op]
        L.append(f"| {op} | {k['avg_ms']*1e3:.1f} | {k['avg_GBps']} | {k['best_ms']*1e3:.1f} |")
    L += ["", f"kernel_source_digest: {digest}", ""]
    open(os.path.join(out, "stream_f64_n2p27_kernel_trace.md"), "w").write("\n".join(L))

    # headline counters
    grid_of = {}
    for (name, g) in cn.vals["FETCH_SIZE"]:
        p = _plain_name(name)
        if p and p[0] == 0:
            grid_of.setdefault(p[1], set()).add(g)
    rows, traffic = [], None
    for op in range(4):
        g = max(grid_of[op])  # the 2^27 launches have the largest grid of their map
        d = cn.launch(rf"stream_kernel<0, {op},", g)
        reads = (ARRAYS[op] - 1) * N27 * 8
        rows.append((OPS[op], d, reads, N27 * 8))
        if op == 3:
            traffic = d["read_bytes"] + d["write_bytes"]
    L = ["# HBM traffic counters: STREAM f64, N = 2^27 per array", "",
         "Four counter runs (each a run of its own), made by `python paper_2206_06302_amd/profiling.py run`:", "",
         *pmc_cmds, "", *calib, "",
         "Per launch of the headline maps (the 2^27 launches of the headline and of the closed-form checks):", "",
         *_traffic_table(rows, ff, fw), "",
         "Read and write requests all reach DRAM (TCC_EA0_RDREQ_DRAM_sum and TCC_EA0_WRREQ_DRAM_sum equal the",
         "totals).  Copy's few extra writes are dirty lines of the preceding triad written back while it runs.",
         "", f"traffic_bytes_per_launch: {traffic:.6e}", f"kernel_source_digest: {digest}", ""]
    open(os.path.join(out, "stream_f64_n2p27_pmc.md"), "w").write("\n".join(L))

    # batched trace
    bb = _bench_json(os.path.join(raw, "trace_batched.json"))["batched"]
    total, tiles, tile = bb["total_elems"], bb["tiles"], bb["tile_elems"]
    cfg = bb["cfg"]
    L = ["# Kernel trace: batched ragged STREAM, 4096 FP64 instances (bench batched leg)", "",
         "Made by `python paper_2206_06302_amd/profiling.py run` (then `summarize`); the run:", "",
         "```", "export TMPDIR=/tmp; cd /tmp", _command(cmds["batched trace"], raw), "```", "",
         f"Batch: 4096 instances, log-uniform lengths in [1e3, 1e7) (seed 5), {total} elements in total,",
         f"{3*total*8/1e9:.1f} GB on the device.  Each map is one launch over all instances: one workgroup",
         f"per group of K consecutive tiles, or P one-wave workgroups per tile, one piece each (the triad's",
         f"plan: {tiles} tiles of {tile} elements, 64-byte tile records).  Triad configuration: block "
         f"{cfg['block']}, U{cfg['unroll']}, {cfg.get('vec_bytes', 16)}-byte vectors, K "
         f"{cfg.get('tiles_per_wg', 1)}, grid/CU {cfg['grid_per_cu']}, nontemporal loads {cfg['nt_load']} and "
         f"stores {cfg['nt_store']}, record read-ahead {cfg.get('record_ahead', 0)}, P {cfg.get('wgs_per_tile', 1)}.",
         "The four-map iteration runs 50 times from a captured graph plus 1 warm-up; then each map runs",
         "alone (1 + 10 launches; the triad 1 + 20).  GB/s = STREAM bytes of one launch / its average duration.", "",
         "| kernel | map | calls | avg ms | min ms | max ms | GB/s (avg) | GB/s (min time) |",
         "|---|---|---|---|---|---|---|---|"]
    for r in _stats(os.path.join(raw, "trace_batched", "run_kernel_stats.csv")):
        m = re.search(r"batch_kernel<(\d+), (\d+), (\d+), (\d+), (\w+), (\w+), (\w+)>", r["Name"])
        mp = re.search(r"batch_piece_kernel<(\d+), (\d+), (\d+), (\w+), (\w+)>", r["Name"])
        if m and m.group(1) == "0":
            op = int(m.group(2))
            name = (f"batch_kernel<f64,{OPS[op]},U{m.group(3)},K{m.group(4)},nt_load={int(m.group(5) == 'true')},"
                    f"nt_store={int(m.group(6) == 'true')},record_ahead={int(m.group(7) == 'true')}>")
        elif mp and mp.group(1) == "0":
            op = int(mp.group(2))
            name = (f"batch_piece_kernel<f64,{OPS[op]},VB{mp.group(3)},nt_load={int(mp.group(4) == 'true')},"
                    f"nt_store={int(mp.group(5) == 'true')}>")
        else:
            continue
        b = ARRAYS[op] * total * 8
        avg, mn, mx = float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"])
        L.append(f"| `{name}` | {OPS[op]} | {r['Calls']} | {avg/1e6:.3f} | {mn/1e6:.3f} | {mx/1e6:.3f} | "
                 f"{b/avg:.1f} | {b/mn:.1f} |")
    L += ["", "From the same run (events on the target's stream, profiler attached):", "",
          f"* graph-replayed four-map iteration: {bb['graph_iteration_ms']} ms ({bb['graph_iteration_GBps']} GB/s)",
          f"* batched triad best {bb['triad_best_GBps']} GB/s, average {bb['triad_avg_GBps']} GB/s; one plain "
          f"launch per instance {bb['plain_per_instance_triad_best_GBps']} GB/s",
          "* each map alone, average GB/s: " + ", ".join(f"{op} {v['avg_GBps']}" for op, v in bb["maps"].items()),
          f"* every element of every instance validated after the replays: {bb['valid_after_graph_replays']}", ""]
    open(os.path.join(out, "batched_f64_4096_kernel_trace.md"), "w").write("\n".join(L))

    # reduced-precision trace
    L = _reduced_summary(raw, _command(cmds["reduced trace"], raw))
    open(os.path.join(out, "stream_reduced_n2p28_kernel_trace.md"), "w").write("\n".join(L))
    if os.path.isdir(os.path.join(raw, "trace_validation")):
        L = _validation_summary(raw, _command(cmds["validation trace"], raw))
        open(os.path.join(out, "checksum_fill_1gib_kernel_trace.md"), "w").write("\n".join(L))

    # batched counters
    bj = _bench_json(os.path.join(raw, "pmc_rdreq.json"))["batched"]
    total, tiles = bj["total_elems"], bj["tiles"]
    rows = []
    for op in range(4):
        d = cn.launch(rf"batch_(?:piece_)?kernel<0, {op},")
        rows.append((OPS[op], d, (ARRAYS[op] - 1) * total * 8, total * 8))
    L = ["# HBM traffic counters: batched ragged STREAM, 4096 FP64 instances", "",
         "Four counter runs (each a run of its own), made by `python paper_2206_06302_amd/profiling.py run`:", "",
         *pmc_cmds, "", *calib, "",
         f"Per launch of each batched map over all {total} elements (dispatches of the captured iteration and",
         "of the maps timed alone).  Each map also reads its tile table: 64 bytes per tile, "
         f"{tiles} tiles of the triad's size ({tiles * 64:.3e} bytes).", "",
         *_traffic_table(rows, ff, fw), "",
         f"traffic_bytes_per_launch (triad): {rows[3][1]['read_bytes'] + rows[3][1]['write_bytes']:.6e}", ""]
    open(os.path.join(out, "batched_f64_4096_pmc.md"), "w").write("\n".join(L))
    print("wrote", ", ".join(sorted(os.listdir(out))))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("action", choices=("run", "summarize"))
    ap.add_argument("--raw", required=True, help="directory of the raw profiler output")
    ap.add_argument("--timeout", type=int, default=300, help="seconds allowed per profiler run")
    ap.add_argument("--out", default=PROFILES, help="directory for the summaries (default: profiles/)")
    a = ap.parse_args()
    if a.action == "run":
        return run(a.raw, a.timeout)
    summarize(a.raw, a.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
