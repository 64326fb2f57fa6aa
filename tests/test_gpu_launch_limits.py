"""Launches past the dispatch's 32-bit count of lanes.  A one-pass launch of
more than 2^32 - 1 lanes would run only part of its grid; the library caps
every grid-stride launch below that count and the kernel's loop covers the
rest.  Elements the launch failed to reach would keep an initial value that
differs from every result, and the last elements are checked against the
oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu

N = (1 << 32) + 9
LANE_LIMIT = (1 << 32) - 1


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    yield ts, torch, tgt
    tgt.synchronize()
    tgt.close()


def _need(torch, nbytes):
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + (2 << 30):
        pytest.skip(f"needs {nbytes / 2 ** 30:.0f} GiB of free device memory")


def test_element_wise_copy_past_the_lane_limit(env):
    """bf16 copy of 2^32 + 9 elements with one element per lane in 1024-lane
    workgroups: one pass would need 2^32 + 1024 lanes."""
    ts, torch, tgt = env
    _need(torch, 2 * 2 * N)
    x = torch.empty(N, dtype=torch.bfloat16, device="cuda")
    d = torch.empty_like(x)
    torch.cuda.synchronize()
    X, D = ts.Array.wrap(tgt, x), ts.Array.wrap(tgt, d)
    X.fill_uniform(11, 0)  # values in [-1, 1]
    D.fill(7.0)
    cfg = {"block": 1024, "unroll": 1, "vec_bytes": 2, "nt_load": 1, "nt_store": 1, "grid_per_cu": 0}
    assert -(-N // 1024) * 1024 > LANE_LIMIT
    say(f"[copy bf16 n={N} block 1024 element-wise]")
    ts.set_kernel_cfg("copy", "bf16", cfg)
    try:
        ts.copy(tgt, X, D)
    finally:
        ts.set_kernel_cfg("copy", "bf16", None)
    assert ts.mismatch_count(tgt, D, X) == 0
    assert torch.equal(d[-64:].cpu(), x[-64:].cpu())
    del X, D, x, d
    torch.cuda.empty_cache()


def test_one_wave_triad_and_transform_past_the_lane_limit(env):
    """The tuned binary64 triad at 2^32 + 9 elements (one-wave workgroups,
    one 8-byte element per lane: one pass would need more than 2^32 lanes)
    and the same triad as a run-time-compiled transform."""
    ts, torch, tgt = env
    _need(torch, 4 * 8 * N)
    x, y, a, d = (torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(4))
    torch.cuda.synchronize()
    X, Y, A, D = (ts.Array.wrap(tgt, t) for t in (x, y, a, d))
    X.fill_uniform(12, 0)
    Y.fill_uniform(12, 1)
    A.fill(7.0)
    D.fill(9.0)
    cfg = ts.get_kernel_cfg("triad", "f64", N)
    per_lane = (cfg["vec_bytes"] // 8) * cfg["unroll"]
    if cfg["grid_per_cu"] == 0:
        assert -(-N // per_lane) > LANE_LIMIT  # the tuned one-pass shape would pass the limit
    say(f"[triad f64 n={N} {cfg}]")
    ts.triad(tgt, X, Y, A, 3.0)
    tr = ts.Transform(tgt, "fma(q, y, x)", 2, "f64")
    try:
        say(f"[transform fma(q, y, x) f64 n={N}]")
        tr(tgt, X, D, Y, 3.0)
        tgt.synchronize()
    finally:
        tr.close()
    assert ts.mismatch_count(tgt, D, A) == 0
    k = 4096
    xs, ys, got = (t[-k:].cpu().numpy() for t in (x, y, a))
    ref = np.empty(k)
    oracle.op(oracle.F64, oracle.OPS["triad"], xs, ys, ref, 3.0)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    del X, Y, A, D, x, y, a, d
    torch.cuda.empty_cache()
