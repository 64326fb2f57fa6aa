"""bench.py's legs at small sizes on the GPU: the headline leg validates in
both copy directions, and the extra legs return well-formed results."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def env():
    import torch

    import bench
    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    yield bench, ts, torch, tgt
    tgt.synchronize()
    tgt.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("order", ["listing", "copy_b"])
def test_main_leg_validates(env, order):
    bench, ts, torch, tgt = env
    m = bench.main_leg(ts, torch, tgt, (1 << 20) + 3, steps=3, warmup=1, order=order)
    assert m["valid"]
    assert set(m["kernels"]) == {"copy", "scale", "add", "triad"}
    assert all(k["best_ms"] > 0 and k["avg_ms"] >= k["best_ms"] for k in m["kernels"].values())


def test_transform_and_overhead_legs(env):
    bench, ts, torch, tgt = env
    t = bench.transform_leg(ts, tgt, 1 << 20, reps=3)
    assert t["same_bits"] and t["avg_ratio"] > 0
    o = bench.overhead_leg(ts, torch, tgt, lo=12, hi=14, iters=32, per_graph=16)
    assert set(o) == {"2^12", "2^14"} and all(r["graph16_us_per_iteration"] > 0 for r in o.values())


def test_reduced_and_calibration_legs(env):
    bench, ts, torch, tgt = env
    r = bench.reduced_leg(ts, torch, tgt, n=(1 << 20) + 5, reps=2, samples=512, chain_steps=3)
    for dtype in ("f64", "f32", "bf16", "f16"):
        for op in ("copy", "scale", "add", "triad"):
            e = r[dtype][op]
            assert e["GBps"] > 0 and e["chain_avg_GBps"] > 0 and e["chain_best_GBps"] >= e["chain_avg_GBps"]
    assert r["f32"]["copy"]["max_rel_err_vs_f64"] == 0.0
    c = bench.calibration_leg(ts, tgt, 1 << 20, reps=2)
    assert c["read_1r"]["bytes_read"] == 8 << 20 and c["write_1w"]["bytes_written"] == 8 << 20
    assert all(c[k]["avg_GBps"] > 0 for k in ("read_1r", "write_1w", "copy_1r1w"))


def test_validation_leg(env):
    bench, ts, torch, tgt = env
    v = bench.validation_leg(ts, tgt, nbytes=(8 << 20) + 48, reps=2)
    assert set(v) == {"f64", "f32", "bf16", "f16"}
    for dt, r in v.items():
        assert r["valid"], dt
        assert r["n"] == ((8 << 20) + 48) // ts.ELEM_SIZE[dt]
        assert r["fill_const_avg_GBps"] > 0 and r["checksum_call_avg_GBps"] > 0 and r["checksum_call_avg_us"] > 0
        assert r["mismatch_call_avg_GBps"] > 0 and r["fill_uniform_avg_GBps"] > 0
