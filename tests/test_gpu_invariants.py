"""Launch-shape invariance: every configuration the tuner may pick (block,
unroll, vector width, nontemporal hints, grid shape; batched tile walk) gives
the oracle's result bit for bit, so tuning can change speed only."""
import numpy as np
import pytest

import oracle
import tsgen
from gpu_util import assert_same_bits, device_array, say

pytestmark = pytest.mark.gpu

OPS = ("copy", "scale", "add", "triad")


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    yield ts, torch, tgt
    for op in OPS:
        for dt in ("f64", "f32", "bf16", "f16"):
            ts.set_kernel_cfg(op, dt, None)
            ts.set_kernel_cfg(op, dt, None, batched=True)
    tgt.synchronize()
    tgt.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("offset", [0, 1])
def test_every_plain_candidate_matches_oracle(env, dtype, offset):
    ts, torch, tgt = env
    n = (1 << 17) + 13
    x = tsgen.uniform_array(31, 0, n, dtype)
    y = tsgen.uniform_array(31, 1, n, dtype)
    X = device_array(ts, torch, tgt, x, dtype, offset)
    Y = device_array(ts, torch, tgt, y, dtype, offset)
    D = device_array(ts, torch, tgt, np.zeros_like(x), dtype, offset)
    cands = ts.candidates()
    for op in OPS:
        ref = np.zeros_like(x)
        oracle.op(oracle.DTYPES[dtype], oracle.OPS[op], x, y if op in ("add", "triad") else None, ref, 3.0)
        R = device_array(ts, torch, tgt, ref, dtype, 0)
        say(f"[invariance {dtype} off={offset} {op}] {len(cands)} candidates")
        for cfg in cands:
            ts.set_kernel_cfg(op, dtype, cfg)
            D.fill(0.0)
            ts.run_op(tgt, op, X, Y, D, 3.0)
            assert ts.mismatch_count(tgt, D, R) == 0, (op, cfg)
        ts.set_kernel_cfg(op, dtype, None)


def test_every_batched_candidate_matches_plain(env):
    ts, torch, tgt = env
    rng = np.random.default_rng(19)
    lens = [0, 1, 7, 9, 1000, 16385, 70001] + list(rng.integers(1, 40000, 9))
    es = 8
    offs, pos = [], 0
    for i, n in enumerate(lens):
        start = (pos + 31) // 32 * 32 + (i % 2)  # every other instance misaligned by one element
        offs.append(start)
        pos = start + int(n)
    init = [torch.from_numpy(tsgen.uniform_array(3, k, pos + 32)).cuda() for k in range(3)]
    work = [t.clone() for t in init]
    ref = [t.clone() for t in init]
    torch.cuda.synchronize()
    qs = tsgen.batched_scalars(2, len(lens))
    mk = lambda pools: [(pools[0].data_ptr() + o * es, pools[1].data_ptr() + o * es, pools[2].data_ptr() + o * es,
                         int(n), float(q)) for o, n, q in zip(offs, lens, qs)]
    bref = ts.Batch(tgt, "f64", mk(ref))
    bw = ts.Batch(tgt, "f64", mk(work))
    for op in OPS:
        bref.op_plain(tgt, op)
    tgt.synchronize()
    cands = ts.candidates(batched=True)
    say(f"[batched invariance] {len(cands)} candidates")
    for cfg in cands:
        for op in OPS:
            ts.set_kernel_cfg(op, "f64", cfg, batched=True)
        bw.set_tile(cfg["tile_elems"])  # the candidate's own tiles
        for k in range(3):
            work[k].copy_(init[k])
        torch.cuda.synchronize()
        for op in OPS:
            bw.op(tgt, op)
        tgt.synchronize()
        for k in range(3):
            assert torch.equal(work[k].view(torch.int64), ref[k].view(torch.int64)), (cfg, k)
    for op in OPS:
        ts.set_kernel_cfg(op, "f64", None, batched=True)
    bref.close(), bw.close()


def test_random_cross_product_matches_oracle(env):
    """300 seeded random cases over storage type x map x size x per-operand
    misalignment x forced launch configuration (any plain candidate), each
    compared with the oracle bit for bit.  Sizes are log-uniform up to 2^20
    so heads, tails and partial last vectors all occur."""
    ts, torch, tgt = env
    rng = np.random.default_rng(2206)
    cands = ts.candidates()
    dtypes, ops = ["f64", "f32", "bf16", "f16"], ["copy", "scale", "add", "triad"]
    try:
        for case in range(300):
            dtype, op = dtypes[rng.integers(4)], ops[rng.integers(4)]
            n = int(np.floor(10 ** rng.uniform(0, 6)))
            offs = tuple(int(v) for v in rng.integers(0, 8, 3))
            cfg = cands[rng.integers(len(cands))]
            q = float(rng.choice([3.0, -0.7, 1e-3, 2.5e4]))
            seed = int(rng.integers(1 << 30))
            ts.set_kernel_cfg(op, dtype, cfg)
            x = tsgen.uniform_array(seed, 0, n, dtype)
            y = tsgen.uniform_array(seed, 1, n, dtype)
            d0 = tsgen.uniform_array(seed, 2, n, dtype)
            X = device_array(ts, torch, tgt, x, dtype, offs[0])
            Y = device_array(ts, torch, tgt, y, dtype, offs[1])
            D = device_array(ts, torch, tgt, d0, dtype, offs[2])
            ts.run_op(tgt, op, X, Y, D, q)
            ref = d0.copy()
            oracle.op(oracle.DTYPES[dtype], oracle.OPS[op], x, y if op in ("add", "triad") else None, ref, q)
            assert_same_bits(D.to_host(), ref, dtype, f"case {case}: {dtype} {op} n={n} offs={offs} cfg={cfg}")
            ts.set_kernel_cfg(op, dtype, None)
    finally:
        for dtype in dtypes:
            for op in ops:
                ts.set_kernel_cfg(op, dtype, None)


def test_autotuner_on_small_problems(env, tmp_path):
    """ts_autotune and ts_autotune_batch time every candidate, keep the
    fastest in the table (which then serves it), and leave results
    unchanged; the table survives a save and load."""
    ts, torch, tgt = env
    cands = ts.candidates()
    try:
        cfg, bps = ts.autotune(tgt, "triad", "f64", (1 << 16) + 7, offset=1, reps=1)
        assert bps > 0 and cfg in cands
        assert ts.get_kernel_cfg("triad", "f64", (1 << 16) + 7, align_class=ts.ALIGN_SHARED) == cfg
        n = (1 << 16) + 7
        x, y = tsgen.uniform_array(31, 0, n), tsgen.uniform_array(31, 1, n)
        X, Y = device_array(ts, torch, tgt, x, "f64", 1), device_array(ts, torch, tgt, y, "f64", 1)
        D = device_array(ts, torch, tgt, np.zeros(n), "f64", 1)
        ts.triad(tgt, X, Y, D, 3.0)
        ref = np.zeros(n)
        oracle.op(oracle.F64, oracle.TRIAD, x, y, ref, 3.0)
        assert_same_bits(D.to_host(), ref, "f64", "after tuning")

        lens = [1000, 5000, 17, 70001, 0, 3]
        offs, pos = [], 0
        for k in lens:
            offs.append((pos + 31) // 32 * 32)
            pos = offs[-1] + k
        pools = [torch.zeros(pos + 64, dtype=torch.float64, device="cuda") for _ in range(3)]
        ref_pools = [torch.zeros(pos + 64, dtype=torch.float64, device="cuda") for _ in range(3)]
        torch.cuda.synchronize()
        mk = lambda p: [(p[0].data_ptr() + o * 8, p[1].data_ptr() + o * 8, p[2].data_ptr() + o * 8, k, 1.5)
                        for o, k in zip(offs, lens)]
        b, r = ts.Batch(tgt, "f64", mk(pools)), ts.Batch(tgt, "f64", mk(ref_pools))
        bcfg, bbps = ts.autotune_batch(tgt, b, "add", reps=1)
        assert bbps > 0 and bcfg in ts.candidates(batched=True)
        assert ts.get_kernel_cfg("add", "f64", sum(lens), batched=True) == bcfg
        for batch in (b, r):
            for k in range(3):
                batch.fill_uniform(tgt, k, 8)
        b.op(tgt, "add")  # the batch re-planned to its own tile, the map to its tuned tile
        r.op_plain(tgt, "add")
        tgt.synchronize()
        assert torch.equal(pools[2].view(torch.int64), ref_pools[2].view(torch.int64))
        b.close(), r.close()

        path = tmp_path / "tuned.json"
        ts.tune_cache_save(str(path))
        ts.tune_cache_clear()
        ts.tune_cache_load(str(path))
        assert ts.get_kernel_cfg("triad", "f64", (1 << 16) + 7, align_class=ts.ALIGN_SHARED) == cfg
        assert ts.get_kernel_cfg("add", "f64", sum(lens), batched=True) == bcfg
    finally:
        ts.tune_cache_clear()
        ts.load_default_tuning()
