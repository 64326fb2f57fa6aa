#!/usr/bin/env python3
"""STREAM benchmark on one MI355X through libtstream (one JSON line on stdout).

Workload (the headline): three binary64 arrays of N = 2^27 elements (1 GiB
each) placed on the GPU by the library's allocator, initialised on the device
to a = 1, b = 2, c = 0, scalar q = 3.  One step = one iteration of the
generic STREAM benchmark (Section 5, Listing 4 of the paper): copy c = a,
scale b = q*c, add c = a + b, triad a = b + q*c, four launches in that order.
W untimed warm-up steps (default 10), then exactly K timed steps (default 20) bracketed by device
synchronisation.  Every launch is bracketed by events on the target's stream,
giving per-kernel best/average times; bytes follow the STREAM convention
(copy and scale move 2 arrays, add and triad 3; GB = 1e9 B).

After timing, the arrays are validated on the GPU: every element of a, b
and c must equal element 0 of its array bit for bit (all elements follow the
same chain), and a separate 10-iteration run from (1, 2, 0) must reproduce
STREAM's closed form a = 15^10, b = 3*15^9, c = 4*15^9 exactly.  Only the
CPU-baseline leg runs the oracle.

Extra legs (skipped with --quick): the batched ragged form (4096 instances,
log-uniform lengths in [1e3, 1e7), one launch per map over all instances,
the iteration captured as a HIP graph and replayed) against per-instance
plain launches; reduced-precision storage (binary32, bfloat16, binary16) at
N = 2^28 per array; a size/alignment sweep from 2^16 to 2^29 elements (L2,
Infinity Cache and HBM regimes); launch overhead at small sizes (eager
calls against HIP graphs); and library comparators on the same traffic (the
runtime's device copy, torch's elementwise b + q*c); and the triad as a
run-time-compiled generic transform; and the validation kernels (constant
fill, checksum) on 1 GiB of each storage type.  --legs picks a subset.  The CPU-baseline leg times the oracle
on host cores.
"""
from __future__ import annotations

import argparse
import importlib.util
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "STREAM Triad/Copy GB/s and % of HBM peak, FP64 N=2^27; batched vs plain"
PEAK_GBPS = 8000.0
OPS = ("copy", "scale", "add", "triad")
EXTRA_LEGS = ("calibration", "ceiling", "batched", "reduced_precision", "sweep", "launch_overhead", "comparators",
              "transform", "validation")
PROFILE_PMC = os.path.join(ROOT, "profiles", "stream_f64_n2p27_pmc.md")


def kernel_source_digest() -> str:
    """Digest of the headline kernels' source and tuned configurations, as
    recorded in the profile summaries (paper_2206_06302_amd/profiling.py,
    loaded by path: it needs neither torch nor the library)."""
    spec = importlib.util.spec_from_file_location(
        "_tstream_profiling", os.path.join(ROOT, "paper_2206_06302_amd", "profiling.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.source_digest(ROOT)


def committed_traffic():
    """HBM bytes per triad launch from the committed rocprofv3 counter runs,
    or None when absent or taken on other kernel sources."""
    if not os.path.exists(PROFILE_PMC):
        return None
    text = open(PROFILE_PMC).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    d = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", text)
    if not m or not d or d.group(1) != kernel_source_digest():
        return None
    return float(m.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _fma(x: float, y: float, z: float) -> float:
    """x*y + z rounded once to binary64 (nearest, ties to even): the exact
    rational value is formed with fractions and divided out by CPython's
    integer true division, which rounds correctly; a finite value beyond the
    largest binary64 rounds to infinity.  Non-finite operands use binary64
    arithmetic directly (its result is then exact)."""
    from fractions import Fraction

    if not (math.isfinite(x) and math.isfinite(y) and math.isfinite(z)):
        return x * y + z
    v = Fraction(x) * Fraction(y) + Fraction(z)
    try:
        return v.numerator / v.denominator
    except OverflowError:
        return math.copysign(math.inf, v)


def exact_chain(a: float, b: float, c: float, q: float, iters: int, order: str = "listing", fused: bool = True):
    """(a, b, c) of one element after `iters` iterations of Listing 4's four
    maps, every operation rounded once to binary64: copy, scale b = q*c (one
    product), add c = a + b (one sum), triad a = b + q*c as one fused
    multiply-add (fused=False rounds the product first: a second rounding,
    which a 50-iteration run from (1, 2, 0) with q = 3 tells apart).  Python
    float products and sums are binary64 operations rounded to nearest even;
    only the fused step needs exact rationals."""
    for _ in range(iters):
        if order == "listing":
            c = a
        else:
            a = b
        b = q * c
        c = a + b
        a = _fma(q, c, b) if fused else b + q * c
    return a, b, c


def chain_check(ts, tgt, arrays, expected) -> bool:
    """Every element of every array equals its expected value bit for bit."""
    return all(ts.checksum(tgt, arr, e)["mismatches"] == 0 for arr, e in zip(arrays, expected))


def fused_chain_check(ts, tgt, A, B, C, iters=50, order="listing") -> bool:
    """A run of `iters` iterations from (1, 2, 0) with q = 3 in the tuned
    launch shapes: every element must equal the exactly rounded chain, whose
    triad rounds once (at 50 iterations an unfused triad differs)."""
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    for _ in range(iters):
        ts.stream_iteration(tgt, A, B, C, 3.0, order=order)
    return chain_check(ts, tgt, (A, B, C), exact_chain(1.0, 2.0, 0.0, 3.0, iters, order))


def main_leg(ts, torch, tgt, n, steps, warmup, order="listing"):
    """Headline: FP64 STREAM at n elements; returns the result dict."""
    A, B, C = (ts.Array.alloc(tgt, "f64", n) for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    tgt.synchronize()
    roles = {"copy": (A, None, C) if order == "listing" else (B, None, A),
             "scale": (C, None, B), "add": (A, B, C), "triad": (B, C, A)}
    ev = [[ts.Event(timing=True) for _ in range(5)] for _ in range(steps)]
    for _ in range(warmup):
        ts.stream_iteration(tgt, A, B, C, 3.0, order=order)
    tgt.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        e = ev[s]
        e[0].record(tgt)
        for k, op in enumerate(OPS):
            x, y, d = roles[op]
            ts.run_op(tgt, op, x, y, d, 3.0)
            e[k + 1].record(tgt)
    tgt.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = {op: [ev[s][k].elapsed_ms(ev[s][k + 1]) for s in range(steps)] for k, op in enumerate(OPS)}
    step_ms = [ev[s][0].elapsed_ms(ev[s][4]) for s in range(steps)]
    # The timed arrays: every element equals the exactly rounded chain after
    # the warm-up and timed steps.  Then a 50-iteration run in the same
    # launch shapes, which an unfused triad would fail.
    valid_timed = chain_check(ts, tgt, (A, B, C), exact_chain(1.0, 2.0, 0.0, 3.0, warmup + steps, order))
    valid_fused = fused_chain_check(ts, tgt, A, B, C, 50, order)
    kernels = {}
    for op in OPS:
        b = ts.stream_bytes(op, n)
        best, avg = min(per[op]), sum(per[op]) / len(per[op])
        kernels[op] = {"bytes": b, "best_ms": round(best, 5), "avg_ms": round(avg, 5),
                       "best_GBps": round(b / best / 1e6, 1), "avg_GBps": round(b / avg / 1e6, 1),
                       "pct_peak_best": round(100 * b / best / 1e6 / PEAK_GBPS, 2),
                       "pct_peak_avg": round(100 * b / avg / 1e6 / PEAK_GBPS, 2),
                       "cfg": ts.get_kernel_cfg(op, "f64", n)}
    for arr in (A, B, C):
        arr.free()
    return {"wall_s": wall, "step_ms": step_ms, "kernels": kernels, "valid": valid_timed and valid_fused,
            "valid_timed_arrays": valid_timed, "valid_k50_fused_chain": valid_fused}


PROBE_KINDS = (("read_1r", 1, 0), ("read_2r", 2, 0), ("write_1w", 0, 1), ("copy_1r1w", 1, 1),
               ("triad_2r1w", 2, 1))
LDS_PER_CU = 160 * 1024  # gfx950


def probe_shapes():
    """Launch shapes the ceiling leg searches for every mix of traffic:
    lanes per workgroup, vectors per lane, their width (16 or 8 bytes, the
    widths the maps use) and layout, nontemporal loads, and a cap on the
    workgroups resident per CU (through dynamic LDS)."""
    shapes = []
    for vb in (16, 8):
        for block in (64, 128, 256, 512, 1024):
            for unroll in (1, 2, 4):
                for wave in ((0,) if unroll == 1 else (0, 1)):
                    for ntl in (0, 1):
                        for cap in (0, 2, 4):
                            lds = 0 if cap == 0 else LDS_PER_CU // cap
                            if cap and (block < 256 or 1024 // block * 2 <= cap):
                                continue  # the cap would not bind, or would leave a CU a few waves
                            shapes.append({"block": block, "unroll": unroll, "vec_bytes": vb, "wave_contiguous": wave,
                                           "nt_load": ntl, "nt_store": 1, "lds_bytes": lds})
    return shapes


def ceiling_leg(ts, tgt, n, reps=20):
    """What the memory system delivers for each mix of traffic, on the
    headline's array size (n binary64 elements per array): the library's
    straight-line probe (ts_probe_bandwidth) reads one or two arrays and
    writes none or one, over a search of launch shapes; per mix, the shape
    with the best average over `reps` launches.  Bytes = arrays touched x
    array bytes, as the STREAM convention counts them.  Then the library's
    four maps in their tuned shapes, each timed alone the same way on the
    same arrays, against the ceiling of their mix."""
    nbytes = 8 * n
    A, B, C = (ts.Array.alloc(tgt, "f64", n) for _ in range(3))
    for k, arr in enumerate((A, B, C)):
        arr.fill_uniform(6, k)
    settle(lambda: ts.run_op(tgt, "triad", A, B, C, 3.0))
    out = {}
    for name, reads, writes in PROBE_KINDS:
        moved = (reads + writes) * nbytes
        ranked = []
        for shape in probe_shapes():
            cfg = dict(shape, reads=reads, writes=writes)
            try:
                ms = timed_launches(ts, tgt, lambda: ts.probe_bandwidth(tgt, cfg, A, B, C, nbytes), reps)
            except ts.TSError as e:
                if "lds_bytes" in str(e):
                    continue  # this device offers less LDS per CU
                raise
            ranked.append((sum(ms) / len(ms), min(ms), shape))
        ranked.sort(key=lambda r: r[0])
        avg, best, shape = ranked[0]
        out[name] = {"avg_GBps": round(moved / avg / 1e6, 1), "best_GBps": round(moved / best / 1e6, 1),
                     "frac_avg": round(moved / avg / 1e6 / PEAK_GBPS, 4), "shape": shape,
                     "runner_up_avg_GBps": [round(moved / r[0] / 1e6, 1) for r in ranked[1:4]],
                     "shapes_tried": len(ranked)}
    # The library's tuned maps timed the same way on the same arrays (each map
    # alone, back to back), against the ceiling of their mix of traffic.
    maps = {}
    for op, x, y, d, ceil in (("copy", A, None, C, "copy_1r1w"), ("scale", A, None, C, "copy_1r1w"),
                              ("add", A, B, C, "triad_2r1w"), ("triad", A, B, C, "triad_2r1w")):
        ms = timed_launches(ts, tgt, lambda: ts.run_op(tgt, op, x, y, d, 3.0), reps)
        moved = ts.stream_bytes(op, n)
        gbps = moved / (sum(ms) / len(ms)) / 1e6
        maps[op] = {"avg_GBps": round(gbps, 1), "vs_ceiling": round(gbps / out[ceil]["avg_GBps"], 4)}
    out["maps_alone"] = maps
    for arr in (A, B, C):
        arr.free()
    return out


CALIBRATION_SHAPE = {"block": 512, "unroll": 1, "vec_bytes": 16, "wave_contiguous": 0, "nt_load": 1, "nt_store": 1,
                     "lds_bytes": 0}


def calibration_leg(ts, tgt, n, reps=3):
    """Probe launches of exactly known traffic, for reading the hardware
    counters: over n binary64 elements per array, the straight-line probe
    reads one array (read_1r), writes one (write_1w), or reads one and writes
    another (copy_1r1w), in one fixed shape.  The read-only probe stores
    nothing unless a lane's fold of its vectors equals a 32-bit mark, which
    seeded uniform data practically never gives.  A profiler run of this leg
    sees these kernels beside the STREAM maps, whose counters they check."""
    nbytes = 8 * n
    A, B, C = (ts.Array.alloc(tgt, "f64", n) for _ in range(3))
    for k, arr in enumerate((A, B, C)):
        arr.fill_uniform(6, k)
    out = {}
    for name, reads, writes in (("read_1r", 1, 0), ("write_1w", 0, 1), ("copy_1r1w", 1, 1)):
        cfg = dict(CALIBRATION_SHAPE, reads=reads, writes=writes)
        ms = timed_launches(ts, tgt, lambda: ts.probe_bandwidth(tgt, cfg, A, B, C, nbytes), reps)
        out[name] = {"bytes_read": reads * nbytes, "bytes_written": writes * nbytes, "launches": reps + 1,
                     "avg_GBps": round((reads + writes) * nbytes / (sum(ms) / len(ms)) / 1e6, 1)}
    out["shape"] = CALIBRATION_SHAPE
    for arr in (A, B, C):
        arr.free()
    return out


def batched_leg(ts, torch, tgt, count=4096, seed=5, replays=50, triad_reps=20, map_reps=10, per_instance=True):
    """Batched ragged STREAM: the graph-captured iteration, each map alone, and
    the triad as one plain launch per instance."""
    import numpy as np

    import tsgen
    lens = tsgen.batched_lengths(seed, count)
    qs = tsgen.batched_scalars(seed, count)
    es = 8
    offs, pos = [], 0
    for n in lens:
        start = (pos + 31) // 32 * 32  # every instance starts on a 256-byte boundary
        offs.append(start)
        pos = start + int(n)
    pools = [torch.empty(pos + 32, dtype=torch.float64, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    descs = [(pools[0].data_ptr() + o * es, pools[1].data_ptr() + o * es, pools[2].data_ptr() + o * es, int(n), float(q))
             for o, n, q in zip(offs, lens, qs)]
    batch = ts.Batch(tgt, "f64", descs)
    total = int(sum(int(n) for n in lens))
    batch.fill(tgt, 0, 1.0), batch.fill(tgt, 1, 2.0), batch.fill(tgt, 2, 0.0)
    tgt.synchronize()
    g = ts.Graph.capture_stream_iteration(tgt, batch)
    e0, e1 = ts.Event(timing=True), ts.Event(timing=True)
    g.launch(tgt, 1)  # warm-up
    e0.record(tgt)
    g.launch(tgt, replays - 1)
    e1.record(tgt)
    e1.synchronize()
    graph_ms = e0.elapsed_ms(e1) / (replays - 1)
    # every element of instance i equals the exactly rounded chain of
    # `replays` iterations from (1, 2, 0) with its own q_i
    expected = [exact_chain(1.0, 2.0, 0.0, float(q), replays) for q in qs]
    exp_cols = [np.array([e[k] for e in expected]) for k in range(3)]

    def chains_hold():
        return all(int(batch.mismatch_count(tgt, k, exp_cols[k]).sum()) == 0 for k in range(3))

    valid = chains_hold()
    # each map alone, one launch over all instances, in listing order: a
    # repeated map recomputes the same result, so the four together make one
    # more iteration of the chain
    maps = {}
    for op, arrays in (("copy", 2), ("scale", 2), ("add", 3), ("triad", 3)):
        ms = timed_launches(ts, tgt, lambda: batch.op(tgt, op), triad_reps if op == "triad" else map_reps)
        mb = arrays * total * es
        maps[op] = {"best_GBps": round(mb / min(ms) / 1e6, 1), "avg_GBps": round(mb / (sum(ms) / len(ms)) / 1e6, 1),
                    "launches": len(ms) + 1, "cfg": ts.get_kernel_cfg(op, "f64", total, batched=True)}
        if op == "triad":
            t_ms = ms
    # comparison: one plain launch per instance (4096 launches per map)
    p_ms = timed_launches(ts, tgt, lambda: batch.op_plain(tgt, "triad"), 5) if per_instance else None
    tb = 3 * total * es
    # the plain triads recompute a from the same b and c: still one iteration past the graph's
    expected = [exact_chain(1.0, 2.0, 0.0, float(q), replays + 1) for q in qs]
    exp_cols = [np.array([e[k] for e in expected]) for k in range(3)]
    valid_after = chains_hold()
    info = batch.info()
    out = {
        "instances": count, "total_elems": total, "device_bytes": 3 * total * es, "tiles": info["tiles"],
        "tile_elems": info["tile_elems"], "valid_after_graph_replays": valid,
        "valid_after_map_launches": valid_after, "graph_replays": replays,
        "graph_iteration_ms": round(graph_ms, 4),
        "graph_iteration_GBps": round(10 * total * es / graph_ms / 1e6, 1),  # 2+2+3+3 arrays per element
        "triad_best_GBps": round(tb / min(t_ms) / 1e6, 1), "triad_avg_GBps": round(tb / (sum(t_ms) / len(t_ms)) / 1e6, 1),
        "plain_per_instance_triad_best_GBps": round(tb / min(p_ms) / 1e6, 1) if p_ms else None,
        "maps": maps,
        "cfg": ts.get_kernel_cfg("triad", "f64", total, batched=True),
    }
    g.close()
    batch.close()
    del pools
    torch.cuda.empty_cache()
    return out


def reduced_leg(ts, torch, tgt, n=1 << 28, reps=10, samples=1 << 14, chain_steps=20):
    """Storage as f64/f32/bf16/f16 (arithmetic in binary32 for the narrow
    types), N = 2^28 per array: per map, GB/s over a chain of 10 + 20
    iterations and over standalone launches, elements/s, and the maximum
    relative error of each map against binary64 arithmetic on the same
    stored inputs (numpy, on sampled elements; normal results only)."""
    import numpy as np

    import tsgen
    out = {}
    rng = np.random.default_rng(4)
    idx = np.unique(rng.integers(0, n, samples))
    tidx = torch.from_numpy(idx).cuda()
    for dtype in ("f64", "f32", "bf16", "f16"):
        tt = [torch.empty(n, dtype=ts.TORCH_DTYPES[dtype], device="cuda") for _ in range(3)]
        torch.cuda.synchronize()
        A, B, C = (ts.Array.wrap(tgt, t) for t in tt)
        A.fill_uniform(4, 0), B.fill_uniform(4, 1), C.fill_uniform(4, 2)
        tgt.synchronize()
        xs = {k: tt[k][tidx].double().cpu().numpy() for k in range(3)}  # exact widening
        roles = {"copy": (A, None, C, 0, None, 2), "scale": (C, None, B, 2, None, 1),
                 "add": (A, B, C, 0, 1, 2), "triad": (B, C, A, 1, 2, 0)}
        res = {}
        # the chain: 10 settling and `chain_steps` timed iterations of the
        # four maps in listing order, per-kernel events (values grow 15-fold
        # per iteration and reach infinity in the 16-bit types; the traffic
        # is the same)
        ev = [[ts.Event(timing=True) for _ in range(5)] for _ in range(chain_steps)]
        settle(lambda: ts.stream_iteration(tgt, A, B, C, 3.0), SETTLE_LAUNCHES // 4)
        for st in range(chain_steps):
            ev[st][0].record(tgt)
            for k, op in enumerate(OPS):
                x, y, d = roles[op][:3]
                ts.run_op(tgt, op, x, y, d, 3.0)
                ev[st][k + 1].record(tgt)
        tgt.synchronize()
        chain = {}
        for k, op in enumerate(OPS):
            ms_list = [ev[st][k].elapsed_ms(ev[st][k + 1]) for st in range(chain_steps)]
            b = ts.stream_bytes(op, n, dtype)
            chain[op] = {"avg_GBps": round(b / (sum(ms_list) / len(ms_list)) / 1e6, 1),
                         "best_GBps": round(b / min(ms_list) / 1e6, 1)}
        # standalone maps from the seeded inputs again
        A.fill_uniform(4, 0), B.fill_uniform(4, 1), C.fill_uniform(4, 2)
        tgt.synchronize()
        for op in OPS:
            x, y, d, ix, iy, idst = roles[op]
            ts.time_op(tgt, op, x, y, d, 3.0, reps=2)
            ms = ts.time_op(tgt, op, x, y, d, 3.0, reps=reps) / reps
            b = ts.stream_bytes(op, n, dtype)
            res[op] = {"GBps": round(b / ms / 1e6, 1), "Gelem_per_s": round(n / ms / 1e6, 2),
                       "chain_avg_GBps": chain[op]["avg_GBps"], "chain_best_GBps": chain[op]["best_GBps"]}
            # one more standalone application from known inputs for the error figure
            for k in range(3):
                tt[k][tidx] = torch.from_numpy(xs[k]).to(tt[k].dtype).cuda()
            torch.cuda.synchronize()
            ts.run_op(tgt, op, x, y, d, 3.0)
            tgt.synchronize()
            got = tt[idst][tidx].double().cpu().numpy()
            xv, yv = xs[ix], (xs[iy] if iy is not None else None)
            ref = {"copy": xv, "scale": 3.0 * xv, "add": xv + (yv if yv is not None else 0),
                   "triad": xv + 3.0 * (yv if yv is not None else 0)}[op]
            tiny = {"f64": 2.0 ** -1022, "f32": 2.0 ** -126, "bf16": 2.0 ** -126, "f16": 2.0 ** -14}[dtype]
            m = np.abs(ref) >= tiny
            res[op]["max_rel_err_vs_f64"] = float(np.max(np.abs(got[m] - ref[m]) / np.abs(ref[m]))) if m.any() else 0.0
            xs = {k: tt[k][tidx].double().cpu().numpy() for k in range(3)}
        out[dtype] = res
        del A, B, C, tt
        torch.cuda.empty_cache()
    for dtype in ("f32", "bf16", "f16"):
        for op in OPS:
            out[dtype][op]["elem_rate_vs_f64"] = round(out[dtype][op]["Gelem_per_s"] / out["f64"][op]["Gelem_per_s"], 2)
    out["n"] = n
    out["error_note"] = ("max relative error of one standalone map vs binary64 arithmetic (numpy) on the "
                         "same stored inputs, over sampled elements with normal results")
    return out


def timed_launches(ts, tgt, launch, reps):
    """Milliseconds of each of `reps` launches enqueued back to back with a
    timing-only event between consecutive ones (after one untimed launch),
    so the device never waits for the host inside a measurement."""
    ev = [ts.Event(timing=True) for _ in range(reps + 1)]
    launch()
    ev[0].record(tgt)
    for i in range(reps):
        launch()
        ev[i + 1].record(tgt)
    ev[-1].synchronize()
    return [ev[i].elapsed_ms(ev[i + 1]) for i in range(reps)]


SETTLE_LAUNCHES = 40


def settle(launch, count=SETTLE_LAUNCHES):
    """Untimed launches before a measurement that follows host-side work
    (compiling, allocating, filling): after the GPU has idled, the first few
    dozen launches of a streaming kernel run up to 20 % slow, then recover."""
    for _ in range(count):
        launch()


def sweep_leg(ts, tgt, lo=16, hi=29, reps=20, b2b_below=22, b2b_reps=100):
    """Size and alignment sweep for f64 and f32 arrays of 2^p elements,
    aligned and as 2^p + 7 elements one element past an aligned base, seeded
    inputs: per map, best and average GB/s over `reps` event-timed launches
    after one warm-up; below 2^b2b_below elements also the rate of
    `b2b_reps` launches between two events (launch-bound sizes).  Regime by
    working set (3 arrays): L2 (<= 32 MiB over 8 XCDs), MALL (<= 256 MiB
    Infinity Cache), else HBM."""
    out = {}
    for dtype in ("f64", "f32"):
        es = ts.ELEM_SIZE[dtype]
        for label, extra, off in (("aligned", 0, 0), ("offset1_plus7", 7, 1)):
            rows = {}
            for p in range(lo, hi + 1):
                n = (1 << p) + extra
                A, B, C = (ts.Array.alloc(tgt, dtype, n, off) for _ in range(3))
                for k, arr in enumerate((A, B, C)):
                    arr.fill_uniform(3, k)
                if p >= 24:
                    settle(lambda: ts.run_op(tgt, "triad", B, C, A, 3.0), SETTLE_LAUNCHES // 2)
                ws = 3 * n * es
                row = {"working_set_MiB": round(ws / 2 ** 20, 2),
                       "regime": "L2" if ws <= 32 << 20 else ("MALL" if ws <= 256 << 20 else "HBM")}
                for op, (x, y, d) in (("copy", (A, None, C)), ("scale", (C, None, B)), ("add", (A, B, C)),
                                      ("triad", (B, C, A))):
                    b = ts.stream_bytes(op, n, dtype)
                    ms = timed_launches(ts, tgt, lambda: ts.run_op(tgt, op, x, y, d, 3.0), reps)
                    row[op + "_GBps"] = round(b / (sum(ms) / len(ms)) / 1e6, 1)
                    row[op + "_best_GBps"] = round(b / min(ms) / 1e6, 1)
                    if p < b2b_below:
                        t = ts.time_op(tgt, op, x, y, d, 3.0, reps=b2b_reps) / b2b_reps
                        row[op + "_b2b_GBps"] = round(b / t / 1e6, 1)
                rows[f"2^{p}"] = row
                for arr in (A, B, C):
                    arr.free()
            out[f"{dtype}_{label}"] = rows
    return out


def overhead_leg(ts, torch, tgt, lo=12, hi=22, iters=192, per_graph=16):
    """Launch overhead at small sizes (the paper's Fig. 5 point: abstraction
    cost shows for small arrays, vanishes for large ones): microseconds per
    four-map iteration issued eagerly through the C ABI from Python, against
    HIP graphs replayed back to back, holding one iteration (4 nodes) or
    `per_graph` iterations each.  A graph launch has a fixed cost that only a
    graph of many nodes amortises."""
    out = {}
    e0, e1 = ts.Event(timing=True), ts.Event(timing=True)

    def per_iteration(run, count):
        run(2)
        e0.record(tgt)
        run(count)
        e1.record(tgt)
        e1.synchronize()
        return 1e3 * e0.elapsed_ms(e1) / iters

    for p in range(lo, hi + 1, 2):
        n = 1 << p
        A, B, C = (ts.Array.alloc(tgt, "f64", n) for _ in range(3))
        A.fill(1.0), B.fill(2.0), C.fill(0.0)

        def eager(k):
            for _ in range(k):
                ts.stream_iteration(tgt, A, B, C, 1.0)

        t_eager = per_iteration(eager, iters)
        g1 = ts.Graph.capture_arrays_iteration(tgt, A, B, C, 1.0)
        t_g1 = per_iteration(lambda k: g1.launch(tgt, k), iters)
        g1.close()
        gk = ts.Graph.capture_arrays_iteration(tgt, A, B, C, 1.0, iterations=per_graph)
        t_gk = per_iteration(lambda k: gk.launch(tgt, k), iters // per_graph)
        gk.close()
        row = {"eager_us_per_iteration": round(t_eager, 2), "graph_us_per_iteration": round(t_g1, 2),
               f"graph{per_graph}_us_per_iteration": round(t_gk, 2)}
        for key, t in (("eager", t_eager), ("graph", t_g1), (f"graph{per_graph}", t_gk)):
            row[f"{key}_GBps"] = round(80 * n / t / 1e3, 1)
        out[f"2^{p}"] = row
        for arr in (A, B, C):
            arr.free()
    return out


def transform_leg(ts, tgt, n, reps=20):
    """The triad as a generic transform: the expression fma(q, y, x) compiled
    at run time (hipRTC) and applied by the library's generic kernels, on
    arrays of the headline's size, against the tuned triad kernel in the same
    run: two rounds in alternating order, reps / 2 launches each.  Both
    results must agree bit for bit."""
    A, B, C, D = (ts.Array.alloc(tgt, "f64", n) for _ in range(4))
    for arr, k in zip((A, B, C), range(3)):
        arr.fill_uniform(2, k)
    D.fill(0.0)
    tr = ts.Transform(tgt, "fma(q, y, x)", 2, "f64")
    cases = (("transform_fma_expression", lambda: tr(tgt, B, D, C, 3.0)),
             ("tuned_triad_kernel", lambda: ts.triad(tgt, B, C, A, 3.0)))
    for _, fn in cases:
        settle(fn, SETTLE_LAUNCHES // 2)
    ms = {name: [] for name, _ in cases}
    for rnd in range(2):
        for name, fn in (cases if rnd == 0 else cases[::-1]):
            ms[name] += timed_launches(ts, tgt, fn, max(1, reps // 2))
    out = {}
    b = ts.stream_bytes("triad", n)
    for name, t in ms.items():
        out[name] = {"best_GBps": round(b / min(t) / 1e6, 1), "avg_GBps": round(b / (sum(t) / len(t)) / 1e6, 1)}
    out["same_bits"] = ts.mismatch_count(tgt, A, D) == 0
    out["avg_ratio"] = round(out["transform_fma_expression"]["avg_GBps"] / out["tuned_triad_kernel"]["avg_GBps"], 3)
    tr.close()
    for arr in (A, B, C, D):
        arr.free()
    return out


def validation_leg(ts, tgt, nbytes=1 << 30, reps=20):
    """The validation kernels on arrays of `nbytes` per storage type: the
    constant and the uniform fill (write only), launch by launch; the
    checksum call (both passes and the copy of its 32-byte result to the
    host; the call waits for it) and the mismatch-count call against a
    second array (two arrays read), each after untimed calls.  GB/s of the
    bytes read or written."""
    out = {}
    for dt in ("f64", "f32", "bf16", "f16"):
        n = nbytes // ts.ELEM_SIZE[dt]
        X = ts.Array.alloc(tgt, dt, n)
        Y = ts.Array.alloc(tgt, dt, n).fill(1.0)

        def fill():
            X.fill(1.0)

        def fill_uniform():
            X.fill_uniform(7, 1)

        def check():
            ts.checksum(tgt, X, 1.0)

        def count():
            ts.mismatch_count(tgt, X, Y)

        settle(fill, SETTLE_LAUNCHES // 2)
        settle(fill_uniform, SETTLE_LAUNCHES // 2)
        tu = timed_launches(ts, tgt, fill_uniform, reps)
        tf = timed_launches(ts, tgt, fill, reps)
        settle(check, 10)
        tc = timed_launches(ts, tgt, check, reps)
        settle(count, 10)
        tm = timed_launches(ts, tgt, count, reps)
        cs = ts.checksum(tgt, X, 1.0)
        same = ts.mismatch_count(tgt, X, Y) == 0
        X.free(), Y.free()
        out[dt] = {"n": n,
                   "fill_const_avg_GBps": round(nbytes / (sum(tf) / len(tf)) / 1e6, 1),
                   "fill_uniform_avg_GBps": round(nbytes / (sum(tu) / len(tu)) / 1e6, 1),
                   "checksum_call_avg_us": round(1e3 * sum(tc) / len(tc), 1),
                   "checksum_call_avg_GBps": round(nbytes / (sum(tc) / len(tc)) / 1e6, 1),
                   "mismatch_call_avg_GBps": round(2 * nbytes / (sum(tm) / len(tm)) / 1e6, 1),
                   "valid": cs["mismatches"] == 0 and cs["sum"] == float(n) and same}
    return out


def comparator_leg(ts, torch, n, reps=20):
    """The same traffic through library kernels, for context, on N binary64
    elements per array: the runtime's device-to-device copy (hipMemcpyAsync
    behind torch's copy_), torch's elementwise b + q*c, and rocBLAS level-1
    routines from the rocBLAS that torch bundles (same HIP runtime):
    daxpy y = a*x + y (two reads, one write, like the triad), dcopy and dscal.
    They run on one stream of their own and are timed with the same kind of
    events as the library's kernels in the headline leg."""
    import ctypes

    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    tgt = ts.Target(0, stream)
    cases = {"runtime_memcpy_d2d": (lambda: z.copy_(x), 16 * n),
             "torch_add_alpha_triad": (lambda: torch.add(x, y, alpha=3.0, out=z), 24 * n)}
    out = {}
    blas, handle = None, ctypes.c_void_p()
    try:
        blas = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "librocblas.so"))
        if blas.rocblas_create_handle(ctypes.byref(handle)) != 0:
            raise RuntimeError("rocblas_create_handle failed")
        blas.rocblas_set_stream(handle, ctypes.c_void_p(stream.cuda_stream))
        alpha = ctypes.c_double(3.0)
        px, py, pz = (ctypes.c_void_p(t.data_ptr()) for t in (x, y, z))
        cases["rocblas_daxpy"] = (lambda: blas.rocblas_daxpy(handle, n, ctypes.byref(alpha), px, 1, py, 1), 24 * n)
        cases["rocblas_dcopy"] = (lambda: blas.rocblas_dcopy(handle, n, px, 1, pz, 1), 16 * n)
        cases["rocblas_dscal"] = (lambda: blas.rocblas_dscal(handle, n, ctypes.byref(alpha), pz, 1), 16 * n)
    except (OSError, AttributeError, RuntimeError) as e:
        out["rocblas"] = {"error": str(e)}
    with torch.cuda.stream(stream):
        settle(cases["runtime_memcpy_d2d"][0])
        for name, (fn, nbytes) in cases.items():
            fn()
            ev = [ts.Event(timing=True) for _ in range(reps + 1)]
            ev[0].record(tgt)
            for i in range(reps):
                fn()
                ev[i + 1].record(tgt)
            ev[-1].synchronize()
            ms = [ev[i].elapsed_ms(ev[i + 1]) for i in range(reps)]
            out[name] = {"best_GBps": round(nbytes / min(ms) / 1e6, 1),
                         "avg_GBps": round(nbytes / (sum(ms) / len(ms)) / 1e6, 1)}
    stream.synchronize()
    if blas is not None and handle.value:
        blas.rocblas_destroy_handle(handle)
    tgt.close()
    del x, y, z
    torch.cuda.empty_cache()
    return out


def host_cpu_info() -> dict:
    """The host's CPU model, sockets and NUMA nodes, and the CPUs this process
    may use, with the physical cores they belong to (SMT siblings share one)."""
    info = {}
    try:
        model, sockets = None, set()
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key = key.strip()
                if key == "model name" and model is None:
                    model = val.strip()
                elif key == "physical id":
                    sockets.add(val.strip())
        info["model"] = model
        info["sockets"] = len(sockets) or None
    except OSError:
        pass
    try:
        info["numa_nodes"] = len([d for d in os.listdir("/sys/devices/system/node")
                                  if d.startswith("node") and d[4:].isdigit()])
    except OSError:
        pass
    allowed = allowed_cpus()
    info["cpus_allowed"] = len(allowed)
    info["cpus_online"] = os.cpu_count()
    cores = set()
    for cpu in allowed:
        topo = f"/sys/devices/system/cpu/cpu{cpu}/topology/"
        try:
            with open(topo + "physical_package_id") as f:
                pkg = f.read().strip()
            with open(topo + "core_id") as f:
                core = f.read().strip()
            cores.add((pkg, core))
        except OSError:
            cores = set()
            break
    if cores:
        info["physical_cores_allowed"] = len(cores)
        info["smt_threads_per_core"] = round(len(allowed) / len(cores), 2)
    return info


def allowed_cpus() -> list:
    try:
        return sorted(os.sched_getaffinity(0))
    except AttributeError:
        return list(range(os.cpu_count() or 1))


def _oracle_timed(oracle, n, threads, target_seconds, max_iters, min_iters=2):
    """Iterations of the oracle's timed mode sized to about target_seconds;
    returns (per-op seconds, final values, iterations, threads used, wall s)."""
    t0 = time.perf_counter()
    secs, _, _ = oracle.stream_timed_f64(n, 1, threads)
    one = float(secs.sum())
    iters = int(max(min_iters, min(max_iters, target_seconds / max(one, 1e-3))))
    secs, fin, used = oracle.stream_timed_f64(n, iters, threads)
    return secs, fin, iters, used, time.perf_counter() - t0


def _rates(secs, n):
    """Aggregate GB/s over the iterations and best GB/s per map (STREAM bytes)."""
    per_iter = secs.sum(axis=1)
    agg = 80 * n / per_iter.mean() / 1e9
    best = {op: round(nb / secs[:, k].min() / 1e9, 2)
            for k, (op, nb) in enumerate(zip(OPS, (16 * n, 16 * n, 24 * n, 24 * n)))}
    return agg, best


def cpu_baseline_leg(n, target_seconds=10.0, single_seconds=3.0, small_n=1 << 20, small_iters=10):
    """The oracle's timed mode on the host (one pinned thread per CPU this
    process may use, first touch): the headline size, the small plain
    configuration (2^20 elements, 10 iterations, checked against STREAM's
    closed form) and one thread at the headline size.  Every run's final
    values must equal the exactly rounded chain."""
    import oracle
    threads = len(allowed_cpus())
    secs, fin, iters, used, spent = _oracle_timed(oracle, n, threads, target_seconds, 300)
    ok = tuple(fin[:3]) == exact_chain(1.0, 2.0, 0.0, 3.0, iters) and tuple(fin[3:]) == tuple(fin[:3])
    agg, best = _rates(secs, n)
    s_secs, s_fin, s_used = oracle.stream_timed_f64(small_n, small_iters, threads)
    s_ok = tuple(s_fin[:3]) == (576650390625.0, 115330078125.0, 153773437500.0) == tuple(s_fin[3:])
    s_agg, s_best = _rates(s_secs, small_n)
    s1, f1, it1, _, spent1 = _oracle_timed(oracle, n, 1, single_seconds, 50)
    ok = ok and tuple(f1[:3]) == exact_chain(1.0, 2.0, 0.0, 3.0, it1)
    return {"value": round(agg, 2), "unit": "GB/s", "cores": used, "kind": "oracle",
            "sample": f"N=2^{n.bit_length()-1} f64 x3 arrays, {iters} iterations of copy/scale/add/triad, "
                      f"{used} pinned threads (one per allowed CPU), first-touch blocks; {spent:.1f} s wall",
            "best_GBps_per_kernel": best,
            "small_n2p20_k10": {"value": round(s_agg, 2), "unit": "GB/s", "threads": s_used,
                                "best_GBps_per_kernel": s_best, "closed_form_exact": bool(s_ok),
                                "regime": "24 MiB working set: host caches"},
            "one_thread": {"value": round(80 * n / s1.sum(axis=1).mean() / 1e9, 2), "unit": "GB/s",
                           "iterations": it1, "wall_s": round(spent1, 1)},
            "host": host_cpu_info(), "valid": bool(ok and s_ok)}


def host_target_leg(ts, n, threads, target_seconds=10.0):
    """STREAM on the library's host-CPU target (pinned workers over equal
    blocks, first-touch bulk construction): the paper's NUMA back-end,
    measured beside the oracle's plain threaded loops on the same cores,
    over a sample of about the same length."""
    cpus = [c for dom in ts.host_numa_domains() for c in dom][:threads]
    tgt = ts.Target.host(cpus)
    A, B, C = (ts.Array.alloc(tgt, "f64", n) for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    roles = {"copy": (A, None, C), "scale": (C, None, B), "add": (A, B, C), "triad": (B, C, A)}
    best = {op: float("inf") for op in OPS}
    t0 = time.perf_counter()
    ts.stream_iteration(tgt, A, B, C, 3.0)  # warm-up
    one = time.perf_counter() - t0
    iters = int(max(2, min(300, target_seconds / max(one, 1e-3))))
    total = 0.0
    for _ in range(iters):
        for op in OPS:
            x, y, d = roles[op]
            ms = ts.time_op(tgt, op, x, y, d, 3.0, reps=1)
            best[op] = min(best[op], ms)
            total += ms
    # the warm-up and the timed iterations follow the exactly rounded chain;
    # then the 50-iteration fused-triad run
    valid = (chain_check(ts, tgt, (A, B, C), exact_chain(1.0, 2.0, 0.0, 3.0, iters + 1))
             and fused_chain_check(ts, tgt, A, B, C, 50))
    for arr in (A, B, C):
        arr.free()
    tgt.close()
    return {"value": round(80 * n * iters / total / 1e6, 2), "unit": "GB/s", "cores": len(cpus),
            "best_GBps_per_kernel": {op: round(ts.stream_bytes(op, n) / best[op] / 1e6, 2) for op in OPS},
            "iterations": iters, "valid": valid}


def metric_records(result: dict) -> list[dict]:
    """One record per measurement of a run, for --jsonl: the workload
    (C2 headline, C3 sweep, C4 reduced precision, C5 batched), map, storage
    type, size, offset, launch configuration, times and rates, and HBM
    counter bytes where committed profiles cover the kernel."""
    import platform

    host = platform.node()
    n = result["config"]["n"]
    recs = []
    traffic = result["roofline"].get("traffic")
    for op, k in result["per_kernel"].items():
        recs.append({"config": "C2", "op": op, "dtype": "f64", "n": n, "offset": 0, "kernel_cfg": k["cfg"],
                     "best_ms": k["best_ms"], "avg_ms": k["avg_ms"], "GBps_best": k["best_GBps"],
                     "GBps_avg": k["avg_GBps"], "pct_peak": k["pct_peak_avg"],
                     "traffic_bytes": traffic if op == "triad" else None, "host": host, "ndev": 1})
    for key, rows in result.get("sweep", {}).items():
        if not isinstance(rows, dict) or "_" not in key:
            continue
        dtype, align = key.split("_", 1)
        for size, row in rows.items():
            if not isinstance(row, dict):
                continue
            p = int(size.split("^")[1])
            for op in OPS:
                if f"{op}_GBps" in row:
                    recs.append({"config": "C3", "op": op, "dtype": dtype, "n": (1 << p) + (0 if align == "aligned" else 7),
                                 "offset": 0 if align == "aligned" else 1, "GBps_avg": row[f"{op}_GBps"],
                                 "GBps_best": row.get(f"{op}_best_GBps"), "regime": row.get("regime"),
                                 "host": host, "ndev": 1})
    for dtype, ops in result.get("reduced_precision", {}).items():
        if not isinstance(ops, dict):
            continue
        for op, row in ops.items():
            if isinstance(row, dict) and "GBps" in row:
                recs.append({"config": "C4", "op": op, "dtype": dtype, "n": 1 << 28, "offset": 0,
                             "GBps_best": row["GBps"], "rel_err_max": row.get("max_rel_err_vs_f64"),
                             "host": host, "ndev": 1})
    b = result.get("batched", {})
    if "triad_best_GBps" in b:
        recs.append({"config": "C5", "op": "triad", "dtype": "f64", "n": b["total_elems"], "offset": 0,
                     "kernel_cfg": b["cfg"], "GBps_best": b["triad_best_GBps"], "GBps_avg": b["triad_avg_GBps"],
                     "instances": b["instances"], "host": host, "ndev": 1})
    return recs


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1 << 27)
    ap.add_argument("--quick", action="store_true", help="headline leg only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--autotune", action="store_true", help="re-tune the four maps before timing")
    ap.add_argument("--legs", type=lambda v: [x for x in v.split(",") if x], default=None,
                    help="comma-separated extra legs to run after the headline (default: all): "
                         + ", ".join(EXTRA_LEGS))
    ap.add_argument("--jsonl", default=None,
                    help="also append one JSON record per measurement to this file")
    ap.add_argument("--no-per-instance", action="store_true",
                    help="batched leg: skip the comparison with one plain launch per instance (keeps "
                         "profiler counter runs small)")
    ap.add_argument("--order", choices=("listing", "copy_b"), default="listing",
                    help="listing: copy c = a (Listing 4); copy_b: the variant with copy a = b")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(STREAM shards with no exchange: each GPU would run the same kernels on its own block).", file=sys.stderr)
        sys.exit(2)
    if a.steps < 1 or a.warmup < 0:
        sys.exit("--steps must be >= 1 and --warmup >= 0")
    if a.legs and set(a.legs) - set(EXTRA_LEGS):
        sys.exit(f"unknown legs: {sorted(set(a.legs) - set(EXTRA_LEGS))}; choose from {', '.join(EXTRA_LEGS)}")

    import torch

    import paper_2206_06302_amd as ts

    stream = torch.cuda.Stream()
    tgt = ts.Target(0, stream)
    info = tgt.info()
    log(f"device: {info['arch']} CUs={info['compute_units']} HBM={info['hbm_bytes']/2**30:.0f} GiB")
    if a.autotune:
        for op in OPS:
            cfg, bps = ts.autotune(tgt, op, "f64", a.n)
            log(f"autotune {op}: {bps/1e9:.1f} GB/s {cfg}")

    log(f"main leg: f64 N={a.n}, warmup={a.warmup}, steps={a.steps}")
    m = main_leg(ts, torch, tgt, a.n, a.steps, a.warmup, a.order)
    if not m["valid"]:
        print("validation failed: the timed arrays or the 50-iteration run differ from the exactly rounded chain",
              file=sys.stderr)
        sys.exit(1)
    k = m["kernels"]
    step_bytes = sum(k[op]["bytes"] for op in OPS)
    ms_per_step = sum(m["step_ms"]) / len(m["step_ms"])
    value = step_bytes / ms_per_step / 1e6
    traffic = committed_traffic()
    tri = k["triad"]
    achieved = tri["bytes"] / tri["avg_ms"] / 1e6
    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "stream_f64_n2^27", "n": a.n, "arrays": 3, "q": 3.0,
                   "init": "a=1,b=2,c=0 (device fill)",
                   "order": "copy c=a,scale,add,triad" if a.order == "listing" else "copy a=b,scale,add,triad",
                   "bytes_per_step": step_bytes},
        "host_wall_ms_per_step": round(1e3 * m["wall_s"] / a.steps, 5),
        "validated": (f"every element of a, b, c after the {a.warmup} + {a.steps} steps equals the exactly rounded "
                      "chain; a 50-iteration run from (1, 2, 0) in the same launch shapes equals the chain with a "
                      "fused triad (an unfused one differs)"),
        "kernel_source_digest": kernel_source_digest(),
        "device": {"arch": info["arch"], "compute_units": info["compute_units"], "hbm_bytes": info["hbm_bytes"]},
        "per_kernel": k,
        "roofline": {"bound": "hbm", "kernel": "triad f64", "achieved": round(achieved, 1), "peak": PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_GBPS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": tri["bytes"]},
    }
    if not a.quick:
        for name, fn in (("calibration", lambda: calibration_leg(ts, tgt, a.n)),
                         ("ceiling", lambda: ceiling_leg(ts, tgt, a.n)),
                         ("batched", lambda: batched_leg(ts, torch, tgt, per_instance=not a.no_per_instance)),
                         ("reduced_precision", lambda: reduced_leg(ts, torch, tgt)),
                         ("sweep", lambda: sweep_leg(ts, tgt)),
                         ("launch_overhead", lambda: overhead_leg(ts, torch, tgt)),
                         ("comparators", lambda: comparator_leg(ts, torch, a.n)),
                         ("transform", lambda: transform_leg(ts, tgt, a.n)),
                         ("validation", lambda: validation_leg(ts, tgt))):
            if a.legs and name not in a.legs:
                continue
            log(f"{name} leg")
            t_leg = time.perf_counter()
            try:
                result[name] = fn()
            except Exception as e:  # an extra leg must not hide the headline
                result[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"{name} leg done in {time.perf_counter() - t_leg:.1f} s")
        if "triad_best_GBps" in result.get("batched", {}):
            bt = result["batched"]
            bt["triad_vs_plain_n2p27_triad"] = round(bt["triad_best_GBps"] / tri["best_GBps"], 3)
            # each batched map against the same map's plain 2^27 launches of this run (averages)
            bt["maps_avg_vs_plain_avg"] = {op: round(v["avg_GBps"] / k[op]["avg_GBps"], 3)
                                           for op, v in bt["maps"].items()}
    if not a.no_cpu:
        log("cpu baseline leg (oracle)")
        try:
            result["cpu_baseline"] = cpu_baseline_leg(a.n)
        except Exception as e:  # the baseline must not hide the headline
            result["cpu_baseline"] = {"error": f"{type(e).__name__}: {e}", "kind": "oracle"}
        if not a.quick and "value" in result["cpu_baseline"]:
            log("host target leg")
            try:
                result["host_target"] = host_target_leg(ts, a.n, result["cpu_baseline"]["cores"])
                result["host_target"]["vs_oracle_threads"] = round(
                    result["host_target"]["value"] / result["cpu_baseline"]["value"], 3)
            except Exception as e:
                result["host_target"] = {"error": f"{type(e).__name__}: {e}"}
    tgt.close()
    result["valid"] = {"timed_arrays": m["valid_timed_arrays"], "k50_fused_chain": m["valid_k50_fused_chain"]}
    result = order_for_output(result)
    if a.jsonl:
        with open(a.jsonl, "a") as f:
            for rec in metric_records(result):
                f.write(json.dumps(rec) + "\n")
    log(summary_text(result["summary"]))
    print(json.dumps(result))


TAIL_KEYS = ("per_kernel", "roofline", "cpu_baseline")


def summary(result: dict) -> dict:
    """The metric's figures in one small object: per-map best and average
    GB/s with % of peak, the ceilings the maps run against, the batched
    triad against the plain one, the graph iteration, the checks and the CPU
    baseline."""
    k = result["per_kernel"]
    s = {op: {"best_GBps": k[op]["best_GBps"], "avg_GBps": k[op]["avg_GBps"], "pct_best": k[op]["pct_peak_best"],
              "pct_avg": k[op]["pct_peak_avg"]} for op in OPS}
    ceil = result.get("ceiling", {})
    if "triad_2r1w" in ceil:
        s["ceiling_avg_GBps"] = {name: ceil[name]["avg_GBps"] for name, _, _ in PROBE_KINDS if name in ceil}
        s["triad_avg_vs_2r1w_ceiling"] = round(k["triad"]["avg_GBps"] / ceil["triad_2r1w"]["avg_GBps"], 4)
        s["copy_avg_vs_1r1w_ceiling"] = round(k["copy"]["avg_GBps"] / ceil["copy_1r1w"]["avg_GBps"], 4)
        if "maps_alone" in ceil:
            s["maps_alone_vs_ceiling"] = {op: v["vs_ceiling"] for op, v in ceil["maps_alone"].items()}
    b = result.get("batched", {})
    if "triad_best_GBps" in b:
        s["batched"] = {"triad_best_GBps": b["triad_best_GBps"], "triad_avg_GBps": b["triad_avg_GBps"],
                        "triad_vs_plain_triad_best": b.get("triad_vs_plain_n2p27_triad"),
                        "graph_iteration_GBps": b["graph_iteration_GBps"],
                        "maps_avg_GBps": {op: v["avg_GBps"] for op, v in b.get("maps", {}).items()},
                        "maps_avg_vs_plain_avg": b.get("maps_avg_vs_plain_avg"),
                        "valid": bool(b["valid_after_graph_replays"] and b["valid_after_map_launches"])}
    s["valid"] = result["valid"]
    cb = result.get("cpu_baseline", {})
    if "value" in cb:
        s["cpu_baseline"] = {"GBps": cb["value"], "threads": cb["cores"], "valid": cb["valid"]}
    return s


def order_for_output(result: dict) -> dict:
    """The JSON line's keys in reading order: the contract's fields, the
    extra legs, then per-kernel figures, roofline, CPU baseline and the
    summary last (the end of the line survives truncation)."""
    out = {key: v for key, v in result.items() if key not in TAIL_KEYS}
    for key in TAIL_KEYS:
        if key in result:
            out[key] = result[key]
    out["summary"] = summary(result)
    return out


def summary_text(s: dict) -> str:
    parts = [f"{op} {s[op]['best_GBps']:.0f}/{s[op]['avg_GBps']:.0f} GB/s best/avg ({s[op]['pct_avg']:.1f}% avg)"
             for op in OPS]
    lines = ["summary: " + "; ".join(parts)]
    if "ceiling_avg_GBps" in s:
        lines.append("ceilings (avg GB/s): " + ", ".join(f"{k} {v:.0f}" for k, v in s["ceiling_avg_GBps"].items())
                     + f"; triad/2r1w {s['triad_avg_vs_2r1w_ceiling']:.3f}, copy/1r1w {s['copy_avg_vs_1r1w_ceiling']:.3f}")
        if "maps_alone_vs_ceiling" in s:
            lines.append("maps alone back to back vs ceiling: " + ", ".join(
                f"{op} {r:.3f}" for op, r in s["maps_alone_vs_ceiling"].items()))
    if "batched" in s:
        b = s["batched"]
        lines.append(f"batched triad {b['triad_best_GBps']:.0f}/{b['triad_avg_GBps']:.0f} GB/s "
                     f"({b['triad_vs_plain_triad_best']}x plain), graph iteration {b['graph_iteration_GBps']:.0f} GB/s, "
                     f"valid {b['valid']}")
        if b.get("maps_avg_vs_plain_avg"):
            lines.append("batched maps avg GB/s (x plain avg): " + ", ".join(
                f"{op} {b['maps_avg_GBps'][op]:.0f} ({r:.3f})" for op, r in b["maps_avg_vs_plain_avg"].items()))
    lines.append(f"valid {s['valid']}")
    if "cpu_baseline" in s:
        lines.append(f"cpu baseline {s['cpu_baseline']['GBps']:.1f} GB/s on {s['cpu_baseline']['threads']} threads")
    return "\n".join(lines)


if __name__ == "__main__":
    main()
