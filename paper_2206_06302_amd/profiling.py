"""rocprofv3 runs of bench.py and the summaries kept under profiles/.

    python paper_2206_06302_amd/profiling.py run --raw DIR        # on a machine with the GPU
    python paper_2206_06302_amd/profiling.py summarize --raw DIR  # anywhere: rewrites profiles/*.md

`run` starts four rocprofv3 runs, each a process of its own with the program
directly after `--`, from /tmp with TMPDIR=/tmp:

  headline trace   --kernel-trace --stats of bench.py --quick --no-cpu --warmup 1 --steps 20
  batched trace    --kernel-trace --stats of bench.py --no-cpu --legs batched --warmup 1 --steps 20
  fetch counters   --pmc FETCH_SIZE of bench.py --no-cpu --legs batched --warmup 1 --steps 3
  write counters   --pmc WRITE_SIZE of the same command

`summarize` turns the raw CSV files into four short markdown summaries: the
per-kernel trace of the headline and of the batched leg (with the bench's own
event timings from the same runs beside rocprof's), and the HBM traffic per
launch of the headline triad and the batched triad.  Counter KiB are scaled
by what the same counters read for the headline copy kernel, which moves
exactly 2^27 x 8 bytes each way.  Each summary records the source digest of
the headline kernels, so the benchmark reports counter traffic only while
the kernels are unchanged.

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


def runs(raw: str) -> list[tuple[str, list[str], str]]:
    """(name, command, stdout file) of the four profiler runs."""
    return [
        ("headline trace", ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv", "-d",
                            os.path.join(raw, "trace_headline"), "-o", "run", "--",
                            *_bench("--quick", "--no-cpu", "--warmup", "1", "--steps", "20")],
         os.path.join(raw, "trace_headline.json")),
        ("batched trace", ["rocprofv3", "--kernel-trace", "--stats", "--output-format", "csv", "-d",
                           os.path.join(raw, "trace_batched"), "-o", "run", "--",
                           *_bench("--no-cpu", "--legs", "batched", "--warmup", "1", "--steps", "20")],
         os.path.join(raw, "trace_batched.json")),
        ("fetch counters", ["rocprofv3", "--pmc", "FETCH_SIZE", "--output-format", "csv", "-d",
                            os.path.join(raw, "pmc_fetch"), "-o", "run", "--",
                            *_bench("--no-cpu", "--legs", "batched", "--warmup", "1", "--steps", "3")],
         os.path.join(raw, "pmc_fetch.json")),
        ("write counters", ["rocprofv3", "--pmc", "WRITE_SIZE", "--output-format", "csv", "-d",
                            os.path.join(raw, "pmc_write"), "-o", "run", "--",
                            *_bench("--no-cpu", "--legs", "batched", "--warmup", "1", "--steps", "3")],
         os.path.join(raw, "pmc_write.json")),
    ]


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


def _plain_name(name):
    m = re.search(r"stream_kernel<(\d+), (\d+), (\d+), (\d+), (\w+), (\w+)>", name)
    if not m:
        return None
    dt, op, vb, u, ntl, nts = m.groups()
    return int(dt), int(op), (f"stream_kernel<f64,{OPS[int(op)]},VB{vb},U{u},nt_load={int(ntl == 'true')},"
                              f"nt_store={int(nts == 'true')}>")


def _short(name):
    m = re.search(r"(\w+_kernel(?:<[^>]*>)?|__amd_rocclr_\w+|reduce_pass2|\w+_pass1<\d+>)", name)
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


def _calibration(fetch, write):
    """Counter scale factors from the headline copy kernel (the largest copy
    grid): it reads and writes exactly 2^27 x 8 bytes."""
    grids = sorted({g for (name, g) in fetch if re.search(r"stream_kernel<0, 0,", name)})
    cf = _pick(fetch, r"stream_kernel<0, 0,", grids[-1])
    cw = _pick(write, r"stream_kernel<0, 0,", grids[-1])
    ff = N27 * 8 / (sum(cf) / len(cf) * 1024)
    fw = N27 * 8 / (sum(cw) / len(cw) * 1024)
    return ff, fw, len(cf), len(cw)


def summarize(raw: str) -> None:
    raw = os.path.abspath(raw)
    digest = source_digest()
    cmds = {name: cmd for name, cmd, _ in runs(raw)}
    fetch = _counters(os.path.join(raw, "pmc_fetch"), "FETCH_SIZE")
    write = _counters(os.path.join(raw, "pmc_write"), "WRITE_SIZE")
    ff, fw, ncf, ncw = _calibration(fetch, write)
    calib = (f"Counter values are KiB per dispatch.  Calibration: the headline copy kernel ({ncf}/{ncw} "
             f"dispatches) reads and writes exactly 2^27 x 8 B, giving the factors fetch x{ff:.4f} and write "
             f"x{fw:.4f}.")
    pmc_cmds = ["```", "export TMPDIR=/tmp; cd /tmp", _command(cmds["fetch counters"], raw),
                _command(cmds["write counters"], raw), "```"]

    # headline trace
    bj = _bench_json(os.path.join(raw, "trace_headline.json"))
    L = ["# Kernel trace: STREAM f64, N = 2^27 per array (bench headline)", "",
         "Made by `python paper_2206_06302_amd/profiling.py run` (then `summarize`); the run:", "",
         "```", "export TMPDIR=/tmp; cd /tmp", _command(cmds["headline trace"], raw), "```", "",
         "31 launches per map (1 warm-up, 20 timed steps, 10 of the closed-form check).  GB/s = STREAM bytes",
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
    open(os.path.join(PROFILES, "stream_f64_n2p27_kernel_trace.md"), "w").write("\n".join(L))

    # headline counters
    grid_of = {}
    for (name, g) in fetch:
        p = _plain_name(name)
        if p and p[0] == 0:
            grid_of.setdefault(p[1], set()).add(g)
    L = ["# HBM traffic counters: STREAM f64, N = 2^27 per array", "",
         "Two counter runs (FETCH_SIZE, then WRITE_SIZE; each a run of its own), made by",
         "`python paper_2206_06302_amd/profiling.py run`:", "", *pmc_cmds, "", calib, "",
         "| map | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetched bytes (scaled) | written bytes (scaled) | "
         "algorithmic read / write bytes | traffic / algorithmic |", "|---|---|---|---|---|---|---|---|"]
    traffic = None
    for op in range(4):
        g = max(grid_of[op])  # the 2^27 launches have the largest grid of their map
        f = _pick(fetch, rf"stream_kernel<0, {op},", g)
        w = _pick(write, rf"stream_kernel<0, {op},", g)
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        fb, wb = fk * 1024 * ff, wk * 1024 * fw
        reads = (ARRAYS[op] - 1) * N27 * 8
        alg = reads + N27 * 8
        L.append(f"| {OPS[op]} | {len(f)}/{len(w)} | {fk:.0f} | {wk:.0f} | {fb:.4e} | {wb:.4e} | "
                 f"{reads:.4e} / {N27*8:.4e} | {(fb+wb)/alg:.4f} |")
        if op == 3:
            traffic = fb + wb
    L += ["", f"traffic_bytes_per_launch: {traffic:.6e}", f"kernel_source_digest: {digest}", ""]
    open(os.path.join(PROFILES, "triad_f64_n2p27_pmc.md"), "w").write("\n".join(L))

    # batched trace
    bb = _bench_json(os.path.join(raw, "trace_batched.json"))["batched"]
    total, tiles, tile = bb["total_elems"], bb["tiles"], bb["tile_elems"]
    cfg = bb["cfg"]
    L = ["# Kernel trace: batched ragged STREAM, 4096 FP64 instances (bench batched leg)", "",
         "Made by `python paper_2206_06302_amd/profiling.py run` (then `summarize`); the run:", "",
         "```", "export TMPDIR=/tmp; cd /tmp", _command(cmds["batched trace"], raw), "```", "",
         f"Batch: 4096 instances, log-uniform lengths in [1e3, 1e7) (seed 5), {total} elements in total,",
         f"{3*total*8/1e9:.1f} GB on the device.  Each map is one launch over all instances, one workgroup",
         f"per tile when grid/CU is 0: {tiles} tiles of {tile} elements (64-byte tile records).  Triad",
         f"configuration: block {cfg['block']}, U{cfg['unroll']}, grid/CU {cfg['grid_per_cu']}, nontemporal "
         f"loads {cfg['nt_load']} and stores {cfg['nt_store']}.",
         "The four-map iteration runs 50 times from a captured graph plus 1 warm-up; the triad also runs",
         "alone (1 + 20 launches).  GB/s = STREAM bytes of one launch / its average duration.", "",
         "| kernel | map | calls | avg ms | min ms | max ms | GB/s (avg) | GB/s (min time) |",
         "|---|---|---|---|---|---|---|---|"]
    for r in _stats(os.path.join(raw, "trace_batched", "run_kernel_stats.csv")):
        m = re.search(r"batch_kernel<(\d+), (\d+), (\d+), (\w+), (\w+)>", r["Name"])
        if not m or m.group(1) != "0":
            continue
        op = int(m.group(2))
        b = ARRAYS[op] * total * 8
        avg, mn, mx = float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"])
        L.append(f"| `batch_kernel<f64,{OPS[op]},U{m.group(3)},nt_load={int(m.group(4) == 'true')},"
                 f"nt_store={int(m.group(5) == 'true')}>` | {OPS[op]} | {r['Calls']} | {avg/1e6:.3f} | "
                 f"{mn/1e6:.3f} | {mx/1e6:.3f} | {b/avg:.1f} | {b/mn:.1f} |")
    L += ["", "From the same run (events on the target's stream, profiler attached):", "",
          f"* graph-replayed four-map iteration: {bb['graph_iteration_ms']} ms ({bb['graph_iteration_GBps']} GB/s)",
          f"* batched triad best {bb['triad_best_GBps']} GB/s, average {bb['triad_avg_GBps']} GB/s; one plain "
          f"launch per instance {bb['plain_per_instance_triad_best_GBps']} GB/s",
          f"* every element of every instance validated after the replays: {bb['valid_after_graph_replays']}", ""]
    open(os.path.join(PROFILES, "batched_f64_4096_kernel_trace.md"), "w").write("\n".join(L))

    # batched counters
    bf, bw = _pick(fetch, r"batch_kernel<0, 3,"), _pick(write, r"batch_kernel<0, 3,")
    fk, wk = sum(bf) / len(bf), sum(bw) / len(bw)
    fetched, written = fk * 1024 * ff, wk * 1024 * fw
    alg_r, alg_w, meta = 2 * total * 8, total * 8, tiles * 64
    L = ["# HBM traffic counters: batched triad, 4096 FP64 instances", "",
         "Two counter runs (FETCH_SIZE, then WRITE_SIZE; each a run of its own), made by",
         "`python paper_2206_06302_amd/profiling.py run`:", "", *pmc_cmds, "", calib, "",
         f"Batched triad (`batch_kernel<f64,triad,...>`, {len(bf)}/{len(bw)} dispatches), {tiles} tiles of "
         f"{tile} elements:", "",
         "| | counter KiB | scaled bytes | algorithmic bytes | ratio |", "|---|---|---|---|---|",
         f"| fetched | {fk:.0f} | {fetched:.4e} | {alg_r:.4e} (b and c) + {meta:.3e} (tile records) | "
         f"{fetched/(alg_r+meta):.4f} |",
         f"| written | {wk:.0f} | {written:.4e} | {alg_w:.4e} (a) | {written/alg_w:.4f} |",
         f"| total | | {fetched+written:.4e} | {alg_r+alg_w:.4e} STREAM bytes | {(fetched+written)/(alg_r+alg_w):.4f} |",
         "", f"The tile records add {meta/(alg_r+alg_w)*100:.2f} % to the STREAM bytes.  Fetches run "
         f"{(fetched/(alg_r+meta)-1)*100:.2f} % above b, c and the",
         f"records together.  In all, HBM traffic per launch is {(fetched+written)/(alg_r+alg_w):.3f}x the STREAM bytes.",
         "", f"traffic_bytes_per_launch: {fetched+written:.6e}", ""]
    open(os.path.join(PROFILES, "batched_triad_f64_4096_pmc.md"), "w").write("\n".join(L))
    print("wrote", ", ".join(sorted(os.listdir(PROFILES))))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("action", choices=("run", "summarize"))
    ap.add_argument("--raw", required=True, help="directory of the raw profiler output")
    ap.add_argument("--timeout", type=int, default=300, help="seconds allowed per profiler run")
    a = ap.parse_args()
    if a.action == "run":
        return run(a.raw, a.timeout)
    summarize(a.raw)
    return 0


if __name__ == "__main__":
    sys.exit(main())
