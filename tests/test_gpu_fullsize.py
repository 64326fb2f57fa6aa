"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses (the committed tuning table).  Every element of every output
array is compared with the oracle: the oracle recomputes the seeded inputs
chunk by chunk on host threads (every output element depends only on the
same element of the inputs), and each device chunk is copied to pinned host
memory and compared bit for bit (gpu_util.compare_whole)."""
import numpy as np
import pytest

import oracle
import tsgen
from gpu_util import compare_whole, mismatches, say, widen

pytestmark = pytest.mark.gpu

N27 = 1 << 27


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    ts.tune_cache_clear()
    ts.load_default_tuning()
    tgt = ts.Target(0, torch.cuda.Stream())
    yield ts, torch, tgt
    tgt.synchronize()
    tgt.close()
    torch.cuda.empty_cache()


def _free(torch):
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _inputs(seed, streams, dtype, s, e):
    """Elements [s, e) of the seeded inputs, narrowed to the storage type."""
    idx = np.arange(s, e, dtype=np.uint64)
    return [tsgen.narrow(tsgen.uniform_pm1(seed, k, idx), dtype) for k in streams]


def test_headline_constant_init_whole_arrays(env):
    """N = 2^27 doubles from (1, 2, 0), q = 3: after 21 and 50 iterations every
    element of a, b, c equals the oracle's recurrence bit for bit (50
    distinguishes a fused triad from an unfused one)."""
    ts, torch, tgt = env
    A, B, C = (ts.Array.alloc(tgt, "f64", N27) for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    say("[headline constant init N=2^27]")
    for k in range(1, 51):
        ts.stream_iteration(tgt, A, B, C, 3.0)
        if k in (1, 13, 21, 50):
            exp = oracle.stream_scalar_f64(1.0, 2.0, 0.0, 3.0, k)
            for arr, e, nm in zip((A, B, C), exp, "abc"):
                cs = ts.checksum(tgt, arr, e)
                assert cs["mismatches"] == 0 and cs["max_abs_dev"] == 0.0, (k, nm, cs)
    for arr in (A, B, C):
        arr.free()
    _free(torch)


def test_headline_random_init_whole_arrays(env):
    """N = 2^27 doubles, all three arrays seeded uniform[-1, 1) (seed 2),
    21 iterations (one warm-up plus 20 timed, as the benchmark runs them):
    every element of a, b and c equals the oracle's chain bit for bit."""
    ts, torch, tgt = env
    tt = [torch.empty(N27, dtype=torch.float64, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    A, B, C = (ts.Array.wrap(tgt, t) for t in tt)
    for k, arr in enumerate((A, B, C)):
        arr.fill_uniform(2, k)
    say("[headline random init N=2^27, 21 iterations, whole arrays]")
    for _ in range(21):
        ts.stream_iteration(tgt, A, B, C, 3.0)
    tgt.synchronize()

    def expected(s, e):
        a, b, c = _inputs(2, (0, 1, 2), "f64", s, e)
        oracle.stream_run(oracle.F64, a, b, c, 3.0, 21)
        return (a, b, c), None

    compare_whole(torch, tt, "f64", expected, N27, "headline random init, 21 iterations")
    del A, B, C, tt
    _free(torch)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("p", [16, 20, 24, 27, 29])
@pytest.mark.parametrize("misaligned", [False, True])
def test_size_sweep(env, dtype, p, misaligned):
    """Sizes 2^p and 2^p + 7 starting one element past an aligned base:
    one iteration of the four maps from seeded inputs, every element of
    a, b and c compared with the oracle."""
    ts, torch, tgt = env
    n = (1 << p) + (7 if misaligned else 0)
    off = 1 if misaligned else 0
    tt = [torch.empty(n + off + 8, dtype=ts.TORCH_DTYPES[dtype], device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    views = [t[off:off + n] for t in tt]
    A, B, C = (ts.Array.wrap(tgt, v) for v in views)
    for k, arr in enumerate((A, B, C)):
        arr.fill_uniform(3, k)
    say(f"[sweep {dtype} 2^{p}{' +7 off1' if misaligned else ''}, whole arrays]")
    ts.stream_iteration(tgt, A, B, C, 3.0)
    tgt.synchronize()

    def expected(s, e):
        a, b, c = _inputs(3, (0, 1, 2), dtype, s, e)
        oracle.stream_run(oracle.DTYPES[dtype], a, b, c, 3.0, 1)
        return (a, b, c), None

    compare_whole(torch, views, dtype, expected, n, f"sweep {dtype} n={n} offset={off}")
    del A, B, C, views, tt
    _free(torch)


# Relative error bound of one standalone map in each storage format: one
# binary32 rounding (unit roundoff 2^-24), then one rounding into the storage
# format (2^-8 for bfloat16, 2^-11 for binary16): (1+e1)(1+e2) - 1.
U32 = 2.0 ** -24
REL_BOUND = {"f32": U32, "bf16": 2.0 ** -8 + U32 + 2.0 ** -8 * U32, "f16": 2.0 ** -11 + U32 + 2.0 ** -11 * U32}
SMALLEST_NORMAL = {"f32": 2.0 ** -126, "bf16": 2.0 ** -126, "f16": 2.0 ** -14}


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_reduced_precision_2p28(env, dtype):
    """N = 2^28 per array in reduced storage: every map standalone equals the
    binary32-math oracle bit for bit at every element, and its relative
    error against binary64 arithmetic on the same stored inputs, over every
    element with a normal result, stays within one rounding of binary32 plus
    one of the storage format (copy: exactly 0)."""
    ts, torch, tgt = env
    n = 1 << 28
    tt = [torch.empty(n, dtype=ts.TORCH_DTYPES[dtype], device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    X, Y, D = (ts.Array.wrap(tgt, t) for t in tt)
    X.fill_uniform(4, 0), Y.fill_uniform(4, 1)
    q32 = float(np.float32(3.0))
    worst = {}
    for op in ("copy", "scale", "add", "triad"):
        say(f"[reduced {dtype} {op} 2^28, whole array]")
        ts.run_op(tgt, op, X, Y, D, 3.0)
        tgt.synchronize()
        two = op in ("add", "triad")

        def expected(s, e, op=op, two=two):
            xs, ys = _inputs(4, (0, 1), dtype, s, e)
            ref = np.zeros_like(xs)
            oracle.op(oracle.DTYPES[dtype], oracle.OPS[op], xs, ys if two else None, ref, 3.0)
            # error of this (bit-identical) result against binary64 arithmetic
            xw, yw = widen(dtype, xs), widen(dtype, ys)
            r64 = np.zeros_like(xw)
            oracle.op(oracle.F64, oracle.OPS[op], xw, yw if two else None, r64, q32)
            normal = np.abs(r64) >= SMALLEST_NORMAL[dtype]
            rel = np.abs(widen(dtype, ref)[normal] - r64[normal]) / np.abs(r64[normal])
            return (ref,), (float(rel.max()) if rel.size else 0.0)

        infos = compare_whole(torch, [tt[2]], dtype, expected, n, f"reduced {dtype} {op}")
        worst[op] = max(infos)
        if op == "copy":
            assert worst[op] == 0.0
        else:
            assert worst[op] <= REL_BOUND[dtype], (op, worst[op])
    print(f"max relative error vs binary64 ({dtype}, every element): {worst}", flush=True)
    del X, Y, D, tt
    _free(torch)


def _batch_expected(seed, lens, qs, first, last, iters, block=1 << 16):
    """The oracle's chains for instances first..last-1 from their seeded
    inputs, each instance's three arrays in element order.  Every element
    evolves alone, so the oracle runs on cache-sized blocks."""
    out = []
    for i in range(first, last):
        n = int(lens[i])
        idx = np.arange(n, dtype=np.uint64)
        a, b, c = (tsgen.uniform_pm1(seed, tsgen.instance_stream(i, k), idx) for k in range(3))
        for s in range(0, n, block):
            oracle.stream_run(oracle.F64, a[s:s + block], b[s:s + block], c[s:s + block], float(qs[i]), iters)
        out.append((a, b, c))
    return out


def test_batched_full_4096_instances(env):
    """The benchmark's batch: 4096 instances, log-uniform lengths in
    [1e3, 1e7) (about 4.2e9 elements, 102 GB), q_i in [0.5, 4).  The captured
    four-map iteration replayed 50 times: from (1, 2, 0) every element of
    instance i equals the scalar chain with q_i; from seeded random inputs
    every element of every instance equals the oracle's chain."""
    import concurrent.futures as cf

    from gpu_util import host_workers

    ts, torch, tgt = env
    count, seed = 4096, 5
    lens = tsgen.batched_lengths(seed, count)
    qs = tsgen.batched_scalars(seed, count)
    offs, pos = [], 0
    for n in lens:
        start = (pos + 31) // 32 * 32
        offs.append(start)
        pos = start + int(n)
    pools = [torch.empty(pos + 32, dtype=torch.float64, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    descs = [(pools[0].data_ptr() + o * 8, pools[1].data_ptr() + o * 8, pools[2].data_ptr() + o * 8, int(n), float(q))
             for o, n, q in zip(offs, lens, qs)]
    batch = ts.Batch(tgt, "f64", descs)
    g = ts.Graph.capture_stream_iteration(tgt, batch)
    batch.fill(tgt, 0, 1.0), batch.fill(tgt, 1, 2.0), batch.fill(tgt, 2, 0.0)
    say(f"[batched 4096 constant init, {batch.info()}]")
    g.launch(tgt, 50)
    exp = [oracle.stream_scalar_f64(1.0, 2.0, 0.0, float(q), 50) for q in qs]
    for k in range(3):
        counts = batch.mismatch_count(tgt, k, [e[k] for e in exp])
        assert int(counts.sum()) == 0, (k, np.nonzero(counts)[0][:8])
    for k in range(3):
        batch.fill_uniform(tgt, k, seed)
    say("[batched 4096 random init, every element]")
    g.launch(tgt, 50)
    tgt.synchronize()
    # groups of consecutive instances of about 2^23 elements, one task each:
    # the oracle's chains, the device range copied to the host, and the
    # bitwise comparison of every element
    groups, first, acc = [], 0, 0
    for i, n in enumerate(lens):
        acc += int(n)
        if acc >= 1 << 23 or i == count - 1:
            groups.append((first, i + 1))
            first, acc = i + 1, 0

    def check(group):
        lo, hi = group
        expected = _batch_expected(seed, lens, qs, lo, hi, 50)
        base, end = offs[lo], offs[hi - 1] + int(lens[hi - 1])
        got = [t[base:end].cpu().numpy() for t in pools]
        for j, i in enumerate(range(lo, hi)):
            s, e = offs[i] - base, offs[i] - base + int(lens[i])
            for k in range(3):
                bad = mismatches(got[k][s:e], expected[j][k], "f64")
                if bad.size:
                    return f"instance {i} array {'abc'[k]}: {bad.size} of {e - s} elements differ, first at {bad[0]}"
        return None

    with cf.ThreadPoolExecutor(host_workers()) as pool:
        for res in pool.map(check, groups):
            assert res is None, res
    g.close()
    batch.close()
    del pools
    _free(torch)


def test_beyond_32bit_element_indices(env):
    """Arrays of more than 2^32 elements (binary16, 8.6 GB each, one element
    past an aligned base) and of 2^31 + 9 binary64 elements: the triad and
    the copy equal the oracle (the generator, for the copy) at every element,
    which covers both sides of 2^31 and 2^32; whole-array checksums agree."""
    ts, torch, tgt = env
    n = (1 << 32) + 37
    bufs = [torch.empty(n + 1, dtype=torch.float16, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    views = [b[1:] for b in bufs]
    X, Y, D = (ts.Array.wrap(tgt, v) for v in views)
    X.fill_uniform(21, 0), Y.fill_uniform(21, 1)
    say("[triad f16 n=2^32+37, whole array]")
    ts.triad(tgt, X, Y, D, 3.0)
    tgt.synchronize()

    def expected_triad(s, e):
        x, y = _inputs(21, (0, 1), "f16", s, e)
        ref = np.zeros_like(x)
        oracle.op(oracle.F16, oracle.TRIAD, x, y, ref, 3.0)
        return (ref,), None

    compare_whole(torch, [views[2]], "f16", expected_triad, n, "triad f16 n=2^32+37")
    X.fill(0.5)
    cs = ts.checksum(tgt, X, 0.5)
    assert cs["mismatches"] == 0 and cs["sum"] == 0.5 * n
    del X, Y, D, views, bufs
    _free(torch)

    n = (1 << 31) + 9
    bufs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    S, T = (ts.Array.wrap(tgt, b) for b in bufs)
    S.fill_uniform(22, 0)
    say("[copy f64 n=2^31+9, whole array]")
    ts.copy(tgt, S, T)
    tgt.synchronize()

    def expected_copy(s, e):
        return (_inputs(22, (0,), "f64", s, e)[0],), None

    compare_whole(torch, [bufs[1]], "f64", expected_copy, n, "copy f64 n=2^31+9")
    assert ts.mismatch_count(tgt, S, T) == 0
    del S, T, bufs
    _free(torch)
