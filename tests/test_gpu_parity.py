"""GPU parity: every map of the STREAM listing (Section 5, Listing 4) through
the C ABI, compared element by element with the CPU oracle on the same
seeded inputs -- bit-exact (0 ulp) in every storage format."""
import numpy as np
import pytest

import oracle
import tsgen
from gpu_util import UINT as UINT_OF, assert_same_bits, device_array, empty_array, say

pytestmark = pytest.mark.gpu

OPS = ("copy", "scale", "add", "triad")
SIZES = [0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 63, 64, 65, 1023, 4096 + 5, (1 << 20), (1 << 20) + 7]


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    stream = torch.cuda.Stream()
    tgt = ts.Target(0, stream)
    yield ts, torch, tgt
    tgt.synchronize()
    tgt.close()
    torch.cuda.empty_cache()


def _inputs(n, dtype, seed=7):
    x = tsgen.uniform_array(seed, 0, n, dtype)
    y = tsgen.uniform_array(seed, 1, n, dtype)
    d0 = tsgen.uniform_array(seed, 2, n, dtype)
    return x, y, d0


def _oracle_op(dtype, op, x, y, d0, q):
    ref = d0.copy()
    oracle.op(oracle.DTYPES[dtype], oracle.OPS[op], x, y if op in ("add", "triad") else None, ref, q)
    return ref


def _run(ts, torch, tgt, op, dtype, x, y, d0, q, offs=(0, 0, 0)):
    X = device_array(ts, torch, tgt, x, dtype, offs[0])
    Y = device_array(ts, torch, tgt, y, dtype, offs[1])
    Dd = device_array(ts, torch, tgt, d0, dtype, offs[2])
    ts.run_op(tgt, op, X, Y, Dd, q)
    return Dd.to_host()


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offset", [0, 1, 3])
def test_f64_ops_zero_ulp(env, op, n, offset):
    ts, torch, tgt = env
    say(f"[f64 {op}] n={n} offset={offset}")
    x, y, d0 = _inputs(n, "f64", seed=11 + n % 5)
    got = _run(ts, torch, tgt, op, "f64", x, y, d0, 3.0, (offset, offset, offset))
    assert_same_bits(got, _oracle_op("f64", op, x, y, d0, 3.0), "f64", f"{op} n={n} off={offset}")


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("offs", [(0, 1, 0), (1, 0, 2), (0, 0, 1), (2, 3, 1)])
def test_f64_mixed_misalignment(env, op, offs):
    ts, torch, tgt = env
    n = (1 << 16) + 13
    say(f"[f64 {op} mixed] offs={offs}")
    x, y, d0 = _inputs(n, "f64", seed=5)
    got = _run(ts, torch, tgt, op, "f64", x, y, d0, 3.0, offs)
    assert_same_bits(got, _oracle_op("f64", op, x, y, d0, 3.0), "f64", f"{op} offs={offs}")


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n,offset", [(1, 0), (7, 1), (17, 3), (1023, 0), ((1 << 20) + 7, 1), ((1 << 18), 0)])
def test_reduced_ops_zero_ulp(env, dtype, op, n, offset):
    ts, torch, tgt = env
    say(f"[{dtype} {op}] n={n} offset={offset}")
    x, y, d0 = _inputs(n, dtype, seed=21)
    for q in (3.0, 0.1):
        got = _run(ts, torch, tgt, op, dtype, x, y, d0, q, (offset, offset, offset))
        assert_same_bits(got, _oracle_op(dtype, op, x, y, d0, q), dtype, f"{dtype} {op} n={n} q={q}")


def _special_values(dtype):
    v = [0.0, -0.0, 1.0, -1.0, 3.0, 0.5, 1e-5, -1e-5, 6e-8, -6e-8, 1e-40, -1e-40, 65504.0, -65504.0,
         70000.0, 3.0e38, -3.0e38, 1.0e-30, np.inf, -np.inf, np.nan, 2.0 ** -24, 2.0 ** -25, 1.5 * 2.0 ** -24]
    if dtype == "f64":
        v += [5e-324, -5e-324, 1.7976931348623157e308, 2.2250738585072014e-308, 1e300, -1e300]
    a = np.array(v, np.float64)
    x = np.repeat(a, a.size)
    y = np.tile(a, a.size)
    return tsgen.narrow(x, dtype), tsgen.narrow(y, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("op", OPS)
def test_special_values(env, dtype, op):
    """Signed zeros, subnormals, overflow to infinity, infinities and NaN,
    every pair, through the vector body and the element-wise paths."""
    ts, torch, tgt = env
    say(f"[special {dtype} {op}]")
    x, y = _special_values(dtype)
    d0 = np.zeros_like(x)
    for q in (3.0, -0.0, 1e-30, 1e30):
        for offs in ((0, 0, 0), (1, 1, 1), (0, 1, 2)):
            got = _run(ts, torch, tgt, op, dtype, x, y, d0, q, offs)
            assert_same_bits(got, _oracle_op(dtype, op, x, y, d0, q), dtype, f"special {dtype} {op} q={q} offs={offs}")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_in_place(env, dtype):
    """dst identical to an input is allowed (in place)."""
    ts, torch, tgt = env
    n = 100003
    x, y, _ = _inputs(n, dtype, seed=3)
    X = device_array(ts, torch, tgt, x, dtype, 1)
    Y = device_array(ts, torch, tgt, y, dtype, 1)
    say(f"[in place {dtype}]")
    ts.triad(tgt, X, Y, X, 3.0)  # x = x + 3*y
    ref = x.copy()
    oracle.op(oracle.DTYPES[dtype], oracle.TRIAD, x.copy(), y, ref, 3.0)
    assert_same_bits(X.to_host(), ref, dtype, "in-place triad")
    ts.scale(tgt, Y, Y, 0.5)
    ref2 = y.copy()
    oracle.op(oracle.DTYPES[dtype], oracle.SCALE, y.copy(), None, ref2, 0.5)
    assert_same_bits(Y.to_host(), ref2, dtype, "in-place scale")


def test_closed_form_c1(env):
    """N = 2^20 doubles from (1, 2, 0), q = 3, ten iterations of Listing 4:
    every element must equal 15^10, 3*15^9, 4*15^9 exactly."""
    ts, torch, tgt = env
    n = 1 << 20
    A, B, C = (empty_array(ts, torch, tgt, n, "f64") for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    say("[closed form N=2^20 K=10]")
    for _ in range(10):
        ts.stream_iteration(tgt, A, B, C, 3.0)
    for arr, exp in ((A, 576650390625.0), (B, 115330078125.0), (C, 153773437500.0)):
        cs = ts.checksum(tgt, arr, exp)
        assert cs["mismatches"] == 0 and cs["max_abs_dev"] == 0.0
        assert cs["sum"] == exp * n  # exact: exp * 2^20 is representable, partial sums exact
    a = np.full(n, 1.0)
    b = np.full(n, 2.0)
    c = np.zeros(n)
    oracle.stream_run(oracle.F64, a, b, c, 3.0, 10)
    assert_same_bits(A.to_host(), a, "f64", "a")
    assert_same_bits(B.to_host(), b, "f64", "b")
    assert_same_bits(C.to_host(), c, "f64", "c")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_iterated_chain_matches_oracle(env, dtype):
    """Random init, 21 iterations in listing order, full-array comparison."""
    ts, torch, tgt = env
    n = (1 << 18) + 3
    a, b, c = _inputs(n, dtype, seed=2)
    A = device_array(ts, torch, tgt, a, dtype)
    B = device_array(ts, torch, tgt, b, dtype)
    C = device_array(ts, torch, tgt, c, dtype)
    say(f"[chain {dtype} K=21]")
    for _ in range(21):
        ts.stream_iteration(tgt, A, B, C, 3.0)
    oracle.stream_run(oracle.DTYPES[dtype], a, b, c, 3.0, 21)
    assert_same_bits(A.to_host(), a, dtype, "a")
    assert_same_bits(B.to_host(), b, dtype, "b")
    assert_same_bits(C.to_host(), c, dtype, "c")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("first", [0, 12345])
def test_fill_uniform_matches_generator(env, dtype, first):
    """Device bulk construction draws the same values as the host generator."""
    ts, torch, tgt = env
    n = (1 << 16) + 5
    A = empty_array(ts, torch, tgt, n, dtype, offset=1)
    say(f"[fill_uniform {dtype} first={first}]")
    A.fill_uniform(9, 2, first)
    ref = tsgen.uniform_array(9, 2, n, dtype, start=first)
    assert_same_bits(A.to_host(), ref, dtype, "fill_uniform")
    A.fill(0.1)
    assert_same_bits(A.to_host(), tsgen.narrow(np.full(n, 0.1), dtype), dtype, "fill")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_fill_small_and_offset(env, dtype):
    """Constant fills store an element-wise head, 8-byte words in 4 KiB
    chunks and an element-wise tail (uniform fills 16-byte vectors): every
    split of n and offset, up to many chunks with a cut one, writes exactly
    [0, n)."""
    ts, torch, tgt = env
    es = ts.ELEM_SIZE[dtype]
    for n in (1, 2, 3, 5, 7, 8, 9, 15, 16, 17, 31, 33, 1000, 4099, 70001):
        for off in range(8):
            buf = torch.empty(n + off + 8, dtype=ts.TORCH_DTYPES[dtype], device="cuda")
            buf.view(torch.uint8).fill_(0x55)
            torch.cuda.synchronize()
            A = ts.Array.wrap(tgt, buf[off:off + n])
            A.fill(-2.5)
            assert_same_bits(A.to_host(), tsgen.narrow(np.full(n, -2.5), dtype), dtype, f"n={n} off={off}")
            raw = buf.view(torch.uint8).cpu().numpy()
            assert np.all(raw[:off * es] == 0x55) and np.all(raw[(off + n) * es:] == 0x55), (n, off)
            A.fill_uniform(17, 3, 1000 + off)
            assert_same_bits(A.to_host(), tsgen.uniform_array(17, 3, n, dtype, start=1000 + off), dtype,
                             f"uniform n={n} off={off}")
            raw = buf.view(torch.uint8).cpu().numpy()
            assert np.all(raw[:off * es] == 0x55) and np.all(raw[(off + n) * es:] == 0x55), (n, off)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("lo,hi", [(0.5, 4.0), (-3.0, 1e-3), (-1.0, 1.0)])
def test_fill_uniform_range_matches_generator(env, dtype, lo, hi):
    """The range form draws the host generator's values; on [-1, 1) it is the
    default fill bit for bit."""
    ts, torch, tgt = env
    n = (1 << 15) + 3
    A = empty_array(ts, torch, tgt, n, dtype)
    say(f"[fill_uniform_range {dtype} [{lo}, {hi})]")
    rc = ts.lib.ts_fill_uniform_range(A.handle, 6, 3, 77, lo, hi)
    assert rc == 0, ts.last_error()
    assert_same_bits(A.to_host(), tsgen.uniform_array(6, 3, n, dtype, start=77, lo=lo, hi=hi), dtype, "range")
    for bad in ((1.0, 1.0), (2.0, 1.0), (float("nan"), 1.0), (0.0, float("inf")), (-1e308, 1e308)):
        assert ts.lib.ts_fill_uniform_range(A.handle, 6, 3, 0, bad[0], bad[1]) == -1


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_checksum_against_oracle(env, dtype):
    ts, torch, tgt = env
    n = (1 << 20) + 11
    x = tsgen.uniform_array(4, 0, n, dtype)
    expected = float(oracle.widen_f64(oracle.DTYPES[dtype], x[100:101])[0])
    X = device_array(ts, torch, tgt, x, dtype)
    say(f"[checksum {dtype}]")
    cs = ts.checksum(tgt, X, expected)
    ref = oracle.checksum(oracle.DTYPES[dtype], x, expected)
    w = oracle.widen_f64(oracle.DTYPES[dtype], x)
    bound = n * 2.0 ** -53 * float(np.abs(w).sum())
    assert abs(cs["sum"] - ref.sum) <= 2 * bound
    dev = np.abs(w - expected)
    assert abs(cs["abs_dev_sum"] - ref.abs_dev_sum) <= 2 * n * 2.0 ** -53 * float(dev.sum())
    assert cs["max_abs_dev"] == ref.max_abs_dev
    assert cs["mismatches"] == ref.mismatches
    # reproducible: the reduction tree depends only on n and the address
    assert ts.checksum(tgt, X, expected) == cs



@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_checksum_many_chunks_per_workgroup(env, dtype):
    """Above 4096 chunks of 16 KiB (64 MiB) every first-pass workgroup of the
    checksum and of the mismatch count takes several chunks, the next one
    loaded while the current one is folded; a size two and a half times
    that, not a whole number of chunks, and an element offset that gives a
    head and a tail, give the oracle's counts and maximum exactly and its
    sums within the summation bound.  The mismatch count compares against a
    copy with bits flipped at the head, chunk edges and the tail, at the
    same offset (chunked path) and at another (element-wise path)."""
    ts, torch, tgt = env
    E = ELEMS_PER_16B[dtype]
    es = 16 // E
    odt = oracle.DTYPES[dtype]
    n = (4096 * 16384 * 2 + 3 * 16384 + 100) // es + 3
    x = tsgen.uniform_array(21, 0, n, dtype)
    w = oracle.widen_f64(odt, x)
    expected = float(w[n // 2])
    ref = oracle.checksum(odt, x, expected)
    bound_sum = 2 * n * 2.0 ** -53 * float(np.abs(w).sum())
    bound_dev = 2 * n * 2.0 ** -53 * float(np.abs(w - expected).sum())
    del w
    r = x.copy()
    chunk = 16384 // es
    plant = sorted({0, 1, chunk - 1, chunk, 4096 * chunk - 1, 4096 * chunk, 4097 * chunk + 5, n - 2, n - 1})
    r.view(UINT_OF[dtype])[plant] ^= 1
    want_mm = oracle.mismatch_count(odt, x, r)
    assert want_mm == len(plant)
    for off in (0, E - 1):
        say(f"[checksum many chunks {dtype} n={n} offset={off}]")
        X = device_array(ts, torch, tgt, x, dtype, off)
        cs = ts.checksum(tgt, X, expected)
        assert cs["mismatches"] == ref.mismatches
        assert cs["max_abs_dev"] == ref.max_abs_dev
        assert abs(cs["sum"] - ref.sum) <= bound_sum
        assert abs(cs["abs_dev_sum"] - ref.abs_dev_sum) <= bound_dev
        for roff in (off, (off + 1) % E):
            say(f"[mismatch many chunks {dtype} n={n} offset={off} ref offset={roff}]")
            R = device_array(ts, torch, tgt, r, dtype, roff)
            assert ts.mismatch_count(tgt, X, R) == want_mm, (off, roff)
            del R
        del X
        torch.cuda.empty_cache()


SPECIAL_BITS = {  # +0, -0, +inf, -inf, two NaN payloads, the smallest subnormal
    "f64": [0x0, 0x8000000000000000, 0x7FF0000000000000, 0xFFF0000000000000,
            0x7FF8000000000001, 0xFFF8000000000ABC, 0x1],
    "f32": [0x0, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00001, 0xFFC00ABC, 0x1],
    "bf16": [0x0, 0x8000, 0x7F80, 0xFF80, 0x7FC1, 0xFFC5, 0x1],
    "f16": [0x0, 0x8000, 0x7C00, 0xFC00, 0x7E01, 0xFE05, 0x1],
}


def _same_or_both_nan(a: float, b: float) -> bool:
    return (np.isnan(a) and np.isnan(b)) or a == b


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_checksum_expected_values(env, dtype):
    """The mismatch test takes one form per expected value: a NaN (elements
    that are NaNs agree, whatever their payloads), +0 or -0 (bits compared,
    so the other zero differs) and any other value (values compared).  An
    array holding signed zeros, infinities, NaNs and subnormals at its head,
    its tail and chunk edges, checked against each kind of expected value,
    gives the oracle's counts and maximum exactly; sums that are not finite
    match exactly, finite ones within the summation bound."""
    ts, torch, tgt = env
    E = ELEMS_PER_16B[dtype]
    odt = oracle.DTYPES[dtype]
    chunk = 16384 // (16 // E)  # elements in one 16 KiB chunk
    n = 3 * chunk + 5
    base = tsgen.uniform_array(23, 0, n, dtype)
    specials = np.array(SPECIAL_BITS[dtype], dtype=UINT_OF[dtype])
    spots = [0, 1, 2, chunk - 1, chunk, chunk + 1, 2 * chunk + 3, n - 7, n - 2, n - 1]
    widened = oracle.widen_f64(odt, base)
    expecteds = [0.0, -0.0, float("nan"), -float("inf"), float("inf"), float(widened[n // 2]), 0.1, 1.5]
    for variant in range(2):
        x = base.copy()
        bits = x.view(UINT_OF[dtype])
        for k, j in enumerate(spots):
            bits[j] = specials[(k + variant) % len(specials)]
        if variant == 1:  # every zero, infinity and NaN kind also in the middle of chunks
            bits[chunk // 2: chunk // 2 + len(specials)] = specials
        w = oracle.widen_f64(odt, x)
        finite = np.isfinite(w)
        for expected in expecteds:
            ref = oracle.checksum(odt, x, expected)
            for off in (0, E - 1):
                say(f"[checksum expected {dtype} variant={variant} expected={expected!r} offset={off}]")
                X = device_array(ts, torch, tgt, x, dtype, off)
                cs = ts.checksum(tgt, X, expected)
                assert cs["mismatches"] == ref.mismatches, (expected, off)
                assert _same_or_both_nan(cs["max_abs_dev"], ref.max_abs_dev), (expected, off)
                for key, got, want, mag in (
                        ("sum", cs["sum"], ref.sum, np.abs(w[finite]).sum()),
                        ("abs_dev_sum", cs["abs_dev_sum"], ref.abs_dev_sum,
                         np.abs(w[finite] - expected).sum() if np.isfinite(expected) else 0.0)):
                    if np.isfinite(want):
                        assert abs(got - want) <= 2 * n * 2.0 ** -53 * float(mag), (key, expected, off)
                    else:
                        assert _same_or_both_nan(got, want), (key, expected, off, got, want)

def test_mismatch_count(env):
    ts, torch, tgt = env
    n = 300001
    x = tsgen.uniform_array(8, 0, n)
    r = x.copy()
    idx = np.array([0, 5, 77777, n - 1])
    r[idx] = np.nextafter(r[idx], 2.0)
    X = device_array(ts, torch, tgt, x, "f64")
    R = device_array(ts, torch, tgt, r, "f64", 1)
    assert ts.mismatch_count(tgt, X, R) == 4
    assert ts.mismatch_count(tgt, X, X) == 0


ELEMS_PER_16B = {"f64": 2, "f32": 4, "bf16": 8, "f16": 8}


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_checksum_and_mismatch_layouts(env, dtype):
    """The reductions read a head up to a 16-byte boundary, 16-byte vectors
    and a tail: every element offset within 16 bytes, sizes below one
    vector, around one 16 KiB chunk for binary64 (2048 elements) and across
    several chunks give the oracle's counts and
    maximum exactly and its sums within the summation bound; the mismatch
    count also takes operands whose offsets differ modulo 16 bytes
    (element-wise path)."""
    ts, torch, tgt = env
    E = ELEMS_PER_16B[dtype]
    odt = oracle.DTYPES[dtype]
    for n in (1, E - 1, E + 1, 2047, 2049, 3 * 2048 + 7, 70001):
        if n < 1:
            continue
        x = tsgen.uniform_array(11, n, n, dtype)
        w = oracle.widen_f64(odt, x)
        expected = float(w[n // 2])
        r = x.copy()
        plant = sorted({0, n // 3, n - 1})
        r.view(UINT_OF[dtype])[plant] ^= 1  # flip the lowest bit
        want_mm = oracle.mismatch_count(odt, x, r)
        assert want_mm == len(plant)
        ref = oracle.checksum(odt, x, expected)
        for off in range(E):
            say(f"[checksum/mismatch {dtype} n={n} offset={off}]")
            X = device_array(ts, torch, tgt, x, dtype, off)
            cs = ts.checksum(tgt, X, expected)
            assert cs["mismatches"] == ref.mismatches
            assert cs["max_abs_dev"] == ref.max_abs_dev
            assert abs(cs["sum"] - ref.sum) <= 2 * n * 2.0 ** -53 * float(np.abs(w).sum())
            assert abs(cs["abs_dev_sum"] - ref.abs_dev_sum) <= 2 * n * 2.0 ** -53 * float(np.abs(w - expected).sum())
            for roff in sorted({off, (off + 1) % E, 0}):
                R = device_array(ts, torch, tgt, r, dtype, roff)
                assert ts.mismatch_count(tgt, X, R) == want_mm, (n, off, roff)
                assert ts.mismatch_count(tgt, R, R) == 0


def test_mismatch_count_nan_payloads(env):
    """Two NaNs agree whatever their payloads; a NaN against a number differs."""
    ts, torch, tgt = env
    n = 5000
    x = tsgen.uniform_array(12, 0, n, "f64")
    r = x.copy()
    xb, rb = x.view(np.uint64), r.view(np.uint64)
    xb[[3, 2500, 4999]] = 0x7ff8000000000001
    rb[[3, 2500, 4999]] = 0xfff8000000000abc
    rb[17] = 0x7ff8000000000000
    X = device_array(ts, torch, tgt, x, "f64")
    R = device_array(ts, torch, tgt, r, "f64")
    assert oracle.mismatch_count(oracle.F64, x, r) == 1
    assert ts.mismatch_count(tgt, X, R) == 1


def test_time_op_and_events(env):
    ts, torch, tgt = env
    n = 1 << 20
    A, B, C = (empty_array(ts, torch, tgt, n, "f64") for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    ms = ts.time_op(tgt, "triad", B, C, A, 3.0, reps=5)
    assert ms > 0
    e0, e1 = ts.Event(), ts.Event()
    e0.record(tgt)
    ts.copy(tgt, A, C)
    e1.record(tgt)
    e1.synchronize()
    assert e1.query() and e0.elapsed_ms(e1) >= 0
    # timing-only events bracket work the same way; results are read after a
    # target synchronisation
    t0, t1 = ts.Event(timing=True), ts.Event(timing=True)
    t0.record(tgt)
    for _ in range(3):
        ts.triad(tgt, B, C, A, 3.0)
    t1.record(tgt)
    t1.synchronize()
    assert t1.query() and t0.elapsed_ms(t1) > 0
    tgt.synchronize()
    assert ts.checksum(tgt, A, 2.0 + 3.0 * 2.0)["mismatches"] == 0  # c = a = 2 after time_op and copy
    done = []
    ts.scale(tgt, C, B, 3.0)
    tgt.then(lambda: done.append(1))
    tgt.synchronize()
    import time
    for _ in range(100):
        if done:
            break
        time.sleep(0.01)
    assert done == [1]


def test_plain_graph_matches_eager(env):
    """A captured iteration replayed K times equals K eager iterations."""
    ts, torch, tgt = env
    n = (1 << 20) + 3
    a, b, c = _inputs(n, "f64", seed=13)
    A1, B1, C1 = (device_array(ts, torch, tgt, v, "f64") for v in (a, b, c))
    A2, B2, C2 = (device_array(ts, torch, tgt, v, "f64", 1) for v in (a, b, c))
    say("[plain graph]")
    g = ts.Graph.capture_arrays_iteration(tgt, A1, B1, C1, 3.0)
    for rep in range(3):
        g.launch(tgt, 2)
        for _ in range(2):
            ts.stream_iteration(tgt, A2, B2, C2, 3.0)
        tgt.synchronize()
        for X, Y, nm in ((A1, A2, "a"), (B1, B2, "b"), (C1, C2, "c")):
            assert ts.mismatch_count(tgt, X, Y) == 0, (rep, nm)
    g.close()
    oracle.stream_run(oracle.F64, a, b, c, 3.0, 6)
    assert_same_bits(A1.to_host(), a, "f64", "a after graph")


@pytest.mark.parametrize("n,offset", [(4099, 1), ((1 << 18) + 5, 3)])
def test_multi_iteration_graph_matches_oracle(env, n, offset):
    """One graph holding 16 iterations (64 nodes), replayed twice with eager
    iterations between the replays, equals the oracle's 34-iteration chain
    from random values, bit for bit."""
    ts, torch, tgt = env
    a, b, c = _inputs(n, "f64", seed=23)
    A, B, C = (device_array(ts, torch, tgt, v, "f64", offset) for v in (a, b, c))
    say(f"[multi-iteration graph] n={n} offset={offset}")
    g = ts.Graph.capture_arrays_iteration(tgt, A, B, C, 3.0, iterations=16)
    g.launch(tgt, 1)
    tgt.synchronize()
    ts.stream_iteration(tgt, A, B, C, 3.0)
    ts.stream_iteration(tgt, A, B, C, 3.0)
    g.launch(tgt, 1)
    tgt.synchronize()
    g.close()
    oracle.stream_run(oracle.F64, a, b, c, 3.0, 34)
    for X, ref, nm in ((A, a, "a"), (B, b, "b"), (C, c, "c")):
        assert_same_bits(X.to_host(), ref, "f64", nm)


@pytest.mark.parametrize("n,offset", [(100003, 1), ((1 << 16) + 8, 0)])
def test_copy_b_variant_matches_oracle(env, n, offset):
    """The variant with copy a = b, from random values, 12 iterations, and
    from (1, 2, 0) against the oracle's pinned integer closed form."""
    ts, torch, tgt = env
    a, b, c = _inputs(n, "f64", seed=29)
    A, B, C = (device_array(ts, torch, tgt, v, "f64", offset) for v in (a, b, c))
    say(f"[copy_b variant] n={n} offset={offset}")
    for _ in range(12):
        ts.stream_iteration(tgt, A, B, C, 3.0, order="copy_b")
    oracle.stream_run_copyb_f64(a, b, c, 3.0, 12)
    for X, ref, nm in ((A, a, "a"), (B, b, "b"), (C, c, "c")):
        assert_same_bits(X.to_host(), ref, "f64", nm)
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    for _ in range(21):
        ts.stream_iteration(tgt, A, B, C, 3.0, order="copy_b")
    s = [np.array([v]) for v in (1.0, 2.0, 0.0)]
    oracle.stream_run_copyb_f64(*s, 3.0, 21)
    for X, ref in zip((A, B, C), s):
        assert ts.checksum(tgt, X, float(ref[0]))["mismatches"] == 0


def test_futures_become_ready_after_the_work(env):
    """A future of the work enqueued so far is made ready by a stream callback
    once that work has finished; its results are then visible to the host."""
    ts, torch, tgt = env
    n = 1 << 24
    A, B, C = (empty_array(ts, torch, tgt, n, "f64") for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    futs = []
    for k in range(6):
        ts.stream_iteration(tgt, A, B, C, 3.0)
        futs.append(tgt.async_())
    futs[-1].wait()
    assert all(f.ready() for f in futs)  # callbacks run in stream order
    a = A.to_host()
    assert np.all(a == 15.0 ** 6)
    pending = []
    for _ in range(3):
        ts.stream_iteration(tgt, A, B, C, 3.0)
        pending.append(tgt.async_())
    for f in pending:  # destroying a pending future waits for its callback
        f.close()
    tgt.synchronize()
    assert ts.checksum(tgt, A, 15.0 ** 9)["mismatches"] == 0


def test_futures_destroyed_as_their_callbacks_run(env):
    """Futures destroyed right after they are made, over short work, so that
    destruction meets the stream callback at every point of its run: each
    destroy returns once the callback is done with the future."""
    ts, torch, tgt = env
    n = 1 << 12
    A, B, C = (empty_array(ts, torch, tgt, n, "f64") for _ in range(3))
    A.fill(1.0), B.fill(2.0), C.fill(0.0)
    for k in range(2000):
        ts.run_op(tgt, "copy", A, None, C, 3.0)
        f = tgt.async_()
        if k % 3 == 0:
            f.wait()
        f.close()
    tgt.synchronize()
    assert ts.checksum(tgt, C, 1.0)["mismatches"] == 0
