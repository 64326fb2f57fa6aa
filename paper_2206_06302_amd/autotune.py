"""Tune launch configurations on this GPU and write the tuning table.

    python -m paper_2206_06302_amd.autotune --out paper_2206_06302_amd/tune/gfx950.json

For every key (map, storage type, size bucket 2^p, alignment class) the
library times each candidate configuration (ts_autotune: block, unroll,
vector width, nontemporal load/store, grid shape) and keeps the fastest; the
batched maps are tuned over a ragged batch of log-uniform lengths
(ts_autotune_batch, which also picks the tile size).  Candidates all give
bit-identical results, so tuning changes speed only.

The table is saved after every size bucket, so an interrupted run loses at
most one bucket; --resume starts from the table at --out and skips every key
it already holds.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--merge", action="store_true", help="start from the existing table at --out")
    ap.add_argument("--resume", action="store_true",
                    help="start from the table at --out and skip the keys it already holds")
    ap.add_argument("--plain", default="f64:16-29,f32:16-29,bf16:26-28,f16:26-28",
                    help="dtype:lo-hi exponent ranges, comma separated")
    ap.add_argument("--ops", default="copy,scale,add,triad")
    ap.add_argument("--aligns", default="0,1", help="alignment classes: 0 aligned, 1 one-element offset")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--batched", type=int, default=4096, help="instances of the batched tuning batch (0: skip)")
    ap.add_argument("--batched-seed", type=int, default=5)
    ap.add_argument("--batched-dtypes", default="f64", help="storage types of the batched tuning, comma separated")
    a = ap.parse_args()

    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    ts.tune_cache_clear()
    done = set()
    if (a.merge or a.resume) and os.path.exists(a.out):
        ts.tune_cache_load(a.out)
        if a.resume:
            for e in json.load(open(a.out)).get("entries", []):
                done.add((e["op"], e["dtype"], int(e["bucket"]), int(e["align"]), int(e["batched"])))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    ops = a.ops.split(",")
    aligns = [int(x) for x in a.aligns.split(",")]
    t0 = time.time()
    for spec in a.plain.split(","):
        if not spec:
            continue
        dtype, rng = spec.split(":")
        lo, hi = (int(x) for x in rng.split("-"))
        for p in range(lo, hi + 1):
            for align in aligns:
                n = (1 << p) + (7 if align == 1 else 0)
                for op in ops:
                    if (op, dtype, p, align, 0) in done:
                        continue
                    cfg, bps = ts.autotune(tgt, op, dtype, n, offset=1 if align == 1 else 0, reps=a.reps)
                    print(f"[{time.time()-t0:7.1f}s] {dtype} {op:5s} 2^{p}{'+7 off1' if align else ''}: "
                          f"{bps/1e9:8.1f} GB/s  {cfg}", flush=True)
            ts.tune_cache_save(a.out)  # checkpoint after every size bucket
    if a.batched:
        import tsgen
        lens = tsgen.batched_lengths(a.batched_seed, a.batched)
        qs = tsgen.batched_scalars(a.batched_seed, a.batched)
        for dtype in a.batched_dtypes.split(","):
            es = ts.ELEM_SIZE[dtype]
            align = 256 // es  # every instance starts on a 256-byte boundary
            offs, pos = [], 0
            for n in lens:
                start = (pos + align - 1) // align * align
                offs.append(start)
                pos = start + int(n)
            pools = [torch.empty(pos + align, dtype=ts.TORCH_DTYPES[dtype], device="cuda") for _ in range(3)]
            torch.cuda.synchronize()
            descs = [(pools[0].data_ptr() + o * es, pools[1].data_ptr() + o * es, pools[2].data_ptr() + o * es,
                      int(n), float(q)) for o, n, q in zip(offs, lens, qs)]
            batch = ts.Batch(tgt, dtype, descs)
            for k in range(3):
                batch.fill_uniform(tgt, k, a.batched_seed)
            bucket = int(batch.info()["total_elems"]).bit_length() - 1
            for op in ops:
                if (op, dtype, bucket, 0, 1) in done:
                    continue
                cfg, bps = ts.autotune_batch(tgt, batch, op, reps=a.reps)
                print(f"[{time.time()-t0:7.1f}s] batched {dtype} {op:5s} {batch.info()['total_elems']} elems: "
                      f"{bps/1e9:8.1f} GB/s  {cfg}", flush=True)
            ts.tune_cache_save(a.out)
            batch.close()
            del pools
            torch.cuda.empty_cache()
    ts.tune_cache_save(a.out)
    print(f"wrote {a.out} after {time.time()-t0:.1f}s", flush=True)
    tgt.close()


if __name__ == "__main__":
    sys.exit(main())
