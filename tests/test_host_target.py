"""The host-CPU target (the paper's NUMA back-end, Section 4.1) through the
C ABI: pinned workers over equal contiguous blocks.  Results must equal the
CPU oracle bit for bit whatever the number of workers; runs without a GPU."""
import numpy as np
import pytest

import oracle
import tsgen

OPS = ("copy", "scale", "add", "triad")
E_UNSUPPORTED, E_SHAPE, E_ALIAS, E_INVALID = -8, -2, -5, -1


@pytest.fixture(scope="module")
def ts():
    import paper_2206_06302_amd as ts
    return ts


def _cpus(ts, k):
    allowed = [c for d in ts.host_numa_domains() for c in d]
    return allowed[:k] if k <= len(allowed) else allowed


@pytest.mark.parametrize("workers", [1, 3, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [0, 1, 2, 7, 1000, 100003])
def test_host_maps_match_oracle(ts, workers, dtype, n):
    tgt = ts.Target.host(_cpus(ts, workers))
    x = tsgen.uniform_array(5, 0, n, dtype)
    y = tsgen.uniform_array(5, 1, n, dtype)
    for op in OPS:
        for q in (3.0, -0.1):
            X = ts.Array.wrap_numpy(tgt, x.copy())
            Y = ts.Array.wrap_numpy(tgt, y.copy())
            D = ts.Array.alloc(tgt, dtype, n).fill(0.0)
            ts.run_op(tgt, op, X, Y, D, q)
            ref = np.zeros_like(x)
            oracle.op(oracle.DTYPES[dtype], oracle.OPS[op], x, y if op in ("add", "triad") else None, ref, q)
            got = D.to_host()
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (op, q)
    tgt.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("offset", [0, 1, 3])
def test_host_maps_large_blocks(ts, dtype, offset):
    """Blocks of 1 MiB and more take the streaming-store path (32-byte
    stores after an element-wise head, element-wise tail): still the
    oracle's results bit for bit, in place too."""
    tgt = ts.Target.host(_cpus(ts, 2))
    n = (1 << 20) + 13
    x = tsgen.uniform_array(14, 0, n, dtype)
    y = tsgen.uniform_array(14, 1, n, dtype)
    for op in OPS:
        X = ts.Array.alloc(tgt, dtype, n, offset)
        X.copy_from_host(x)
        Y = ts.Array.alloc(tgt, dtype, n, offset)
        Y.copy_from_host(y)
        D = ts.Array.alloc(tgt, dtype, n, offset)
        D.fill(0.0)
        ts.run_op(tgt, op, X, Y, D, -1.25)
        ref = np.zeros_like(x)
        oracle.op(oracle.DTYPES[dtype], oracle.OPS[op], x, y if op in ("add", "triad") else None, ref, -1.25)
        assert np.array_equal(D.to_host().view(np.uint8), ref.view(np.uint8)), op
        ts.run_op(tgt, op, X, Y, X, -1.25)  # in place
        assert np.array_equal(X.to_host().view(np.uint8), ref.view(np.uint8)), (op, "in place")
    tgt.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_host_fill_large_blocks(ts, dtype):
    """Large-block constant fills (streaming stores) write exactly the
    array, at every offset, with the value's exact bits."""
    tgt = ts.Target.host(_cpus(ts, 3))
    n = (1 << 20) + 5
    for off in range(4):
        A = ts.Array.alloc(tgt, dtype, n, off)
        A.fill(-0.0)
        A.fill(-2.5)
        got = A.to_host()
        assert np.all(got == -2.5), off
        A.fill(-0.0)
        assert np.all(np.signbit(A.to_host())), off
    tgt.close()


@pytest.mark.parametrize("workers", [1, 5])
def test_host_iteration_matches_oracle_chain(ts, workers):
    """Random init, 50 iterations (the fused-triad detector length)."""
    tgt = ts.Target.host(_cpus(ts, workers))
    n = 65539
    arrs = [ts.Array.alloc(tgt, "f64", n, offset=1) for _ in range(3)]
    for k, arr in enumerate(arrs):
        arr.fill_uniform(2, k)
    for _ in range(50):
        ts.stream_iteration(tgt, *arrs, 3.0)
    host = [tsgen.uniform_array(2, k, n) for k in range(3)]
    oracle.stream_run(oracle.F64, host[0], host[1], host[2], 3.0, 50)
    for arr, ref in zip(arrs, host):
        assert np.array_equal(arr.to_host().view(np.uint64), ref.view(np.uint64))
    tgt.close()


def test_host_closed_form_and_checksum(ts):
    tgt = ts.Target.host()
    n = 1 << 20
    A, B, C = (ts.Array.alloc(tgt, "f64", n) for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    for _ in range(10):
        ts.stream_iteration(tgt, A, B, C, 3.0)
    for arr, e in zip((A, B, C), (576650390625.0, 115330078125.0, 153773437500.0)):
        cs = ts.checksum(tgt, arr, e)
        assert cs["mismatches"] == 0 and cs["max_abs_dev"] == 0.0
        assert abs(cs["sum"] - e * n) <= n * 2.0 ** -53 * e * n  # rounding of the block sums
    x = tsgen.uniform_array(9, 0, 12345)
    X = ts.Array.wrap_numpy(tgt, x)
    cs = ts.checksum(tgt, X, float(x[7]))
    ref = oracle.checksum(oracle.F64, x, float(x[7]))
    assert cs["mismatches"] == ref.mismatches and cs["max_abs_dev"] == ref.max_abs_dev
    assert abs(cs["sum"] - ref.sum) <= x.size * 2.0 ** -53 * float(np.abs(x).sum())
    r = x.copy()
    r[[0, 100, 12344]] += 1.0
    assert ts.mismatch_count(tgt, X, ts.Array.wrap_numpy(tgt, r)) == 3
    tgt.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_host_fill_uniform_matches_generator(ts, dtype):
    tgt = ts.Target.host(_cpus(ts, 3))
    A = ts.Array.alloc(tgt, dtype, 100001)
    A.fill_uniform(7, 2, 99)
    assert np.array_equal(A.to_host().view(np.uint8), tsgen.uniform_array(7, 2, 100001, dtype, start=99).view(np.uint8))
    tgt.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("lo,hi", [(0.5, 4.0), (-3.0, 1e-3)])
def test_host_fill_uniform_range_matches_generator(ts, dtype, lo, hi):
    tgt = ts.Target.host(_cpus(ts, 4))
    A = ts.Array.alloc(tgt, dtype, 70001)
    A.fill_uniform(8, 1, 5, lo=lo, hi=hi)
    ref = tsgen.uniform_array(8, 1, 70001, dtype, start=5, lo=lo, hi=hi)
    assert np.array_equal(A.to_host().view(np.uint8), ref.view(np.uint8))
    for bad in ((1.0, 1.0), (2.0, 1.0), (float("nan"), 1.0), (-float("inf"), 0.0), (-1e308, 1e308)):
        with pytest.raises(ts.TSError) as e:
            A.fill_uniform(8, 1, lo=bad[0], hi=bad[1])
        assert e.value.status == E_INVALID
    tgt.close()


def test_host_target_limits(ts):
    tgt = ts.Target.host(_cpus(ts, 2))
    with pytest.raises(ts.TSError) as e:
        ts.Array.alloc(tgt, "bf16", 10).fill(1.0)
    assert e.value.status == E_UNSUPPORTED
    a, b = ts.Array.alloc(tgt, "f64", 100), ts.Array.alloc(tgt, "f64", 99)
    with pytest.raises(ts.TSError) as e:
        ts.copy(tgt, a, b)
    assert e.value.status == E_SHAPE
    c = ts.Array.alloc(tgt, "f64", 100)
    a.fill(5.0), c.fill(7.0)
    with pytest.raises(ts.TSError) as e:  # scale would not fit b: nothing runs
        ts.stream_iteration(tgt, a, b, c)
    assert e.value.status == E_SHAPE and np.all(c.to_host() == 7.0)
    with pytest.raises(ts.TSError) as e:
        ts.Graph.capture_arrays_iteration(tgt, a, a, a)
    assert e.value.status == E_UNSUPPORTED
    with pytest.raises(ts.TSError) as e:
        ts.Graph.capture_arrays_iteration(tgt, a, a, a, iterations=8)
    assert e.value.status == E_UNSUPPORTED
    with pytest.raises(ts.TSError) as e:
        ts.Batch(tgt, "f64", [])
    assert e.value.status == E_UNSUPPORTED
    with pytest.raises(ts.TSError) as e:
        ts.autotune(tgt, "triad", "f64", 1000)
    assert e.value.status == E_UNSUPPORTED
    with pytest.raises(ts.TSError):
        ts.Event().record(tgt)
    with pytest.raises(ts.TSError):
        tgt.stream_handle()
    with pytest.raises(ts.TSError):
        ts.Target.host([100000])
    with pytest.raises(ts.TSError) as e:
        ts.Transform(tgt, "x + 1", 1, "bf16")
    assert e.value.status == E_UNSUPPORTED
    with pytest.raises(ts.TSError) as e:
        ts.copy(tgt, ts.Array.alloc(tgt, "u8", 10), ts.Array.alloc(tgt, "u8", 10))
    assert e.value.status == E_UNSUPPORTED
    done = []
    tgt.then(lambda: done.append(1))
    assert done == [1]
    f = tgt.async_()
    assert f.ready()
    f.wait()
    ms = ts.time_op(tgt, "triad", a, a, a, 3.0, reps=3)
    assert ms >= 0
    tgt.close()


TO_UPPER = "(x >= 'a' && x <= 'z') ? x - ('a' - 'A') : x"


@pytest.mark.parametrize("workers", [1, 4])
def test_host_transforms(ts, workers):
    """Generic transforms on a host target (compiled by the system C++
    compiler, run by the pinned workers): the hello-world to_upper over
    bytes, the fused triad against the oracle, and a general expression
    against numpy's IEEE evaluation."""
    tgt = ts.Target.host(_cpus(ts, workers))
    text = b"hello world"
    s = ts.Array.wrap_numpy(tgt, np.frombuffer(text, np.uint8).copy())
    up = ts.Transform(tgt, TO_UPPER, 1, "u8")
    up(tgt, s, s)  # in place, Listing 3
    assert s.to_host().tobytes() == b"HELLO WORLD"
    n = 100003
    x = tsgen.uniform_array(12, 0, n)
    y = tsgen.uniform_array(12, 1, n)
    X, Y = ts.Array.wrap_numpy(tgt, x.copy()), ts.Array.wrap_numpy(tgt, y.copy())
    D = ts.Array.alloc(tgt, "f64", n)
    tr = ts.Transform(tgt, "fma(q, y, x)", 2, "f64")
    tr(tgt, X, D, Y, 3.0)
    ref = np.zeros(n)
    oracle.op(oracle.F64, oracle.TRIAD, x, y, ref, 3.0)
    assert np.array_equal(D.to_host().view(np.uint64), ref.view(np.uint64))
    g = ts.Transform(tgt, "x * x - q * y", 2, "f64")
    g(tgt, X, D, Y, 0.75)
    assert np.array_equal(D.to_host().view(np.uint64), (x * x - 0.75 * y).view(np.uint64))
    xf, yf = tsgen.uniform_array(12, 0, n, "f32"), tsgen.uniform_array(12, 1, n, "f32")
    XF, YF = ts.Array.wrap_numpy(tgt, xf.copy()), ts.Array.wrap_numpy(tgt, yf.copy())
    DF = ts.Array.alloc(tgt, "f32", n)
    f = ts.Transform(tgt, "x + y", 2, "f32")
    f(tgt, XF, DF, YF)
    ref32 = np.zeros_like(xf)
    oracle.op(oracle.F32, oracle.ADD, xf, yf, ref32, 0.0)
    assert np.array_equal(DF.to_host().view(np.uint32), ref32.view(np.uint32))
    for t_ in (up, tr, g, f):
        t_.close()
    tgt.close()


def test_host_transform_errors(ts):
    tgt = ts.Target.host(_cpus(ts, 2))
    with pytest.raises(ts.TSError) as e:
        ts.Transform(tgt, "x +* y", 2, "f64")
    assert e.value.status == E_INVALID and "error" in e.value.message
    with pytest.raises(ts.TSError) as e:  # y is not defined for one input
        ts.Transform(tgt, "x + y", 1, "f64")
    assert e.value.status == E_INVALID
    tr = ts.Transform(tgt, "x + 1.0", 1, "f64")
    a, short = ts.Array.alloc(tgt, "f64", 100), ts.Array.alloc(tgt, "f64", 99)
    with pytest.raises(ts.TSError) as e:
        tr(tgt, a, short)
    assert e.value.status == E_SHAPE
    with pytest.raises(ts.TSError) as e:
        tr(tgt, ts.Array.alloc(tgt, "f32", 100), ts.Array.alloc(tgt, "f32", 100))
    assert e.value.status == -3
    tr.close()
    tgt.close()
