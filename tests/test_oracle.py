"""Pins of the CPU oracle against facts fixed outside it.

* the closed form of the benchmark iteration from (1, 2, 0) with q = 3
  (Section 5, Listing 4: c = a, b = 3a, c = 4a, a = 15a per iteration);
* exact rational brute force, rounded once (tests/exact.py), on tiny random
  arrays for every op and storage type, including signed zeros, subnormals
  and overflow;
* the fused triad: at 50 iterations the chain's value differs between one
  rounding and two, and the oracle must give the one-rounding value.
"""
import math
import os

import numpy as np
import pytest

import exact
import tsgen

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

OPS = ("copy", "scale", "add", "triad")


# ---------------------------------------------------------------- closed form
@pytest.mark.parametrize("k", list(range(0, 14)))
def test_closed_form_f64(oracle_lib, k):
    """From (1, 2, 0) with q = 3 one iteration maps a to 15a, b to 3a, c to
    4a; all values stay integers below 2^53 up to k = 13, so they are exact."""
    o = oracle_lib
    n = 37
    a = np.full(n, 1.0)
    b = np.full(n, 2.0)
    c = np.full(n, 0.0)
    o.stream_run(o.F64, a, b, c, 3.0, k)
    if k == 0:
        exp = (1.0, 2.0, 0.0)
    else:
        exp = (float(15 ** k), float(3 * 15 ** (k - 1)), float(4 * 15 ** (k - 1)))
    assert np.all(a == exp[0]) and np.all(b == exp[1]) and np.all(c == exp[2])


def test_closed_form_ten_iterations_values(oracle_lib):
    a, b, c = oracle_lib.stream_scalar_f64(1.0, 2.0, 0.0, 3.0, 10)
    assert (a, b, c) == (576650390625.0, 115330078125.0, 153773437500.0)


@pytest.mark.parametrize("k", [14, 21, 33, 50, 51, 80])
def test_long_chain_matches_exact_rounding(oracle_lib, k):
    """Beyond 15^13 the chain rounds; each step must be one correctly rounded
    IEEE operation, the triad a single rounding."""
    got = oracle_lib.stream_scalar_f64(1.0, 2.0, 0.0, 3.0, k)
    ref = exact.stream_scalar(1.0, 2.0, 0.0, 3.0, k, "f64", fused=True)
    assert [exact.f64_bits(v) for v in got] == [exact.f64_bits(v) for v in ref]


def test_fused_triad_is_detectable_at_50(oracle_lib):
    """The one-rounding and two-rounding chains part at 50 iterations, so the
    constant-init run detects an unfused triad; the oracle is the fused one."""
    fused = exact.stream_scalar(1.0, 2.0, 0.0, 3.0, 50, "f64", fused=True)
    unfused = exact.stream_scalar(1.0, 2.0, 0.0, 3.0, 50, "f64", fused=False)
    assert exact.f64_bits(fused[0]) != exact.f64_bits(unfused[0])
    got = oracle_lib.stream_scalar_f64(1.0, 2.0, 0.0, 3.0, 50)
    assert exact.f64_bits(got[0]) == exact.f64_bits(fused[0])
    # relative deviation from the exact 15^50 stays near one unit roundoff
    assert abs(got[0] - 15.0 ** 50) / 15.0 ** 50 < 1e-15


# ------------------------------------------- variant with copy a <- b
def _binet_copyb(k):
    """Closed form of the variant from (1, 2, 0) with q = 3.  One iteration
    maps (a, b, c) to (3b + 12c, 3c, b + 3c), so c follows
    c[k+1] = 3c[k] + 3c[k-1] with c[0] = 0, c[1] = 2, whose solution is
    c[k] = 2 (l1^k - l2^k) / sqrt(21), l1,2 = (3 +- sqrt(21)) / 2; then
    b[k] = 3c[k-1] and a[k] = b[k] + 3c[k].  Evaluated in 60-digit decimal
    arithmetic and rounded to the nearest integer."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    r = Decimal(21).sqrt()
    l1, l2 = (3 + r) / 2, (3 - r) / 2

    def cc(j):
        return int((2 * (l1 ** j - l2 ** j) / r).to_integral_value())
    c = cc(k)
    b = 3 * cc(k - 1)
    return b + 3 * c, b, c


@pytest.mark.parametrize("k", [1, 2, 5, 10, 21, 25])
def test_copyb_variant_closed_form(oracle_lib, k):
    exp = _binet_copyb(k)
    assert max(exp) < 2 ** 53  # exact in binary64
    n = 19
    a, b, c = np.full(n, 1.0), np.full(n, 2.0), np.full(n, 0.0)
    oracle_lib.stream_run_copyb_f64(a, b, c, 3.0, k)
    assert np.all(a == exp[0]) and np.all(b == exp[1]) and np.all(c == exp[2])


def test_copyb_variant_ten_iterations_values():
    assert _binet_copyb(10) == (1015254, 211896, 267786)


def test_copyb_variant_random_matches_exact_ops(oracle_lib):
    """Random operands, 3 iterations, every step an exactly rounded IEEE
    operation (exact rational arithmetic, rounded once)."""
    rng = np.random.default_rng(31)
    n = 9
    a, b, c = (_random_f64(rng, n) for _ in range(3))
    q = -1.3
    ra, rb, rc = a.copy(), b.copy(), c.copy()
    oracle_lib.stream_run_copyb_f64(a, b, c, q, 3)
    for j in range(n):
        x, y, z = float(ra[j]), float(rb[j]), float(rc[j])
        for _ in range(3):
            x = y
            y = exact.mul(q, z, "f64")
            z = exact.add(x, y, "f64")
            x = exact.fma(q, z, y, "f64")
        assert _same(a[j], x) and _same(b[j], y) and _same(c[j], z), j


# -------------------------------------------------------- brute force (f64)
def _special_f64():
    return np.array([0.0, -0.0, 1.0, -1.0, 5e-324, -5e-324, 2.2250738585072014e-308,
                     1.7976931348623157e308, -1.7976931348623157e308, 0.5, 3.0,
                     1.0000000000000002, -0.9999999999999999, 1e-300, 1e300], np.float64)


def _random_f64(rng, n):
    # full 53-bit significands across a wide exponent range, both signs
    mant = rng.random(n) + 1.0
    exp = rng.integers(-60, 60, n)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return sign * np.ldexp(mant, exp)


def _ref_op_f64(op, x, y, q):
    if op == "copy":
        return x
    if op == "scale":
        return exact.mul(q, x, "f64")
    if op == "add":
        return exact.add(x, y, "f64")
    return exact.fma(q, y, x, "f64")


def _same(a: float, b: float) -> bool:
    if math.isnan(a) and math.isnan(b):
        return True
    return exact.f64_bits(a) == exact.f64_bits(b)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 8, 17, 64])
def test_bruteforce_f64(oracle_lib, op, n):
    o = oracle_lib
    rng = np.random.default_rng(1000 + n * 7 + OPS.index(op))
    x = _random_f64(rng, n)
    y = _random_f64(rng, n)
    for q in (3.0, -0.7071067811865476, float(rng.random() * 4)):
        dst = np.full(n, np.nan)
        o.op(o.F64, o.OPS[op], x, y, dst, q)
        for j in range(n):
            assert _same(dst[j], _ref_op_f64(op, x[j], y[j], q)), (op, j, x[j], y[j], q)


@pytest.mark.parametrize("op", OPS)
def test_bruteforce_f64_special_pairs(oracle_lib, op):
    """Every pair of special values, both orders: signed zeros, subnormals,
    the largest finite value (overflow to infinity), exact cancellation."""
    o = oracle_lib
    s = _special_f64()
    x = np.repeat(s, s.size)
    y = np.tile(s, s.size)
    for q in (3.0, -1.0, 0.0, -0.0, 2.0 ** -1074, 1e300):
        dst = np.empty_like(x)
        o.op(o.F64, o.OPS[op], x, y, dst, q)
        for j in range(x.size):
            assert _same(dst[j], _ref_op_f64(op, x[j], y[j], q)), (op, x[j], y[j], q, dst[j])


# ----------------------------------------------- brute force (reduced storage)
def _widen(o, dtype, arr):
    return o.widen_f64(o.DTYPES[dtype], arr)


def _ref_lowp(op, x, y, q, dtype):
    """Widen (exact), evaluate in binary32 with q rounded once to binary32,
    then round the binary32 result once more into the storage format."""
    if op == "copy":
        return x
    q32 = exact.narrow(q, "f32")
    if op == "scale":
        r = exact.mul(q32, x, "f32")
    elif op == "add":
        r = exact.add(x, y, "f32")
    else:
        r = exact.fma(q32, y, x, "f32")
    return exact.narrow(r, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
@pytest.mark.parametrize("op", OPS)
def test_bruteforce_reduced(oracle_lib, dtype, op):
    o = oracle_lib
    rng = np.random.default_rng(77 + OPS.index(op))
    n = 64
    wide = np.concatenate([rng.uniform(-1, 1, n), rng.uniform(-70000, 70000, 8),
                           np.array([0.0, -0.0, 6e-8, -3e-8, 1e-40, 65504.0, 3.0e38, 1.0, -2.0])])
    # storage inputs as the generator narrows them (binary32 first, then RNE)
    x = tsgen.narrow(wide, dtype)
    y = tsgen.narrow(wide[::-1].copy(), dtype)
    xw = _widen(o, dtype, x)
    yw = _widen(o, dtype, y)
    for q in (3.0, 0.1, -2.5):
        dst = np.zeros_like(x)
        o.op(o.DTYPES[dtype], o.OPS[op], x, y, dst, q)
        dw = _widen(o, dtype, dst)
        for j in range(x.size):
            ref = _ref_lowp(op, float(xw[j]), float(yw[j]), q, dtype)
            assert _same(float(dw[j]), ref), (dtype, op, j, xw[j], yw[j], q, dw[j], ref)


@pytest.mark.parametrize("dtype,k", [("f32", 6), ("f32", 7), ("f32", 20), ("f32", 33),
                                     ("bf16", 3), ("bf16", 9), ("f16", 3), ("f16", 5)])
def test_reduced_chain_matches_exact(oracle_lib, dtype, k):
    """Constant-init chain in reduced storage: every step a binary32 op then
    one narrowing; binary16 overflows to infinity after a few iterations."""
    o = oracle_lib
    a = tsgen.narrow(np.full(5, 1.0), dtype)
    b = tsgen.narrow(np.full(5, 2.0), dtype)
    c = tsgen.narrow(np.full(5, 0.0), dtype)
    o.stream_run(o.DTYPES[dtype], a, b, c, 3.0, k)
    ra, rb, rc = 1.0, 2.0, 0.0
    for _ in range(k):
        rc = ra
        rb = _ref_lowp("scale", rc, None, 3.0, dtype)
        rc = _ref_lowp("add", ra, rb, 3.0, dtype)
        ra = _ref_lowp("triad", rb, rc, 3.0, dtype)
    for arr, ref in ((a, ra), (b, rb), (c, rc)):
        w = _widen(o, dtype, arr)
        assert all(_same(float(v), ref) for v in w), (dtype, k, w[0], ref)
    if dtype == "f32" and k == 6:
        assert ra == 11390625.0  # 15^6 < 2^24: still exact
    if dtype == "f16" and k == 5:
        assert math.isinf(ra)    # 15^5 * ... exceeds 65504


# ------------------------------------------------------------- converters
EXHAUSTIVE = os.environ.get("TS_EXHAUSTIVE") == "1"


def _structured_f32_patterns(seed: int) -> np.ndarray:
    """Every upper-16-bit pattern (sign, exponent, top fraction bits) combined
    with every rounding class of the lower bits: zero, one, and one below, at
    and above each half-way point a narrowing to bfloat16 or binary16 can use
    (bits 12..15), plus the all-ones pattern; then 2^25 random patterns."""
    lows = {0, 1, 0xFFFF}
    for h in (0x1000, 0x2000, 0x4000, 0x8000):
        lows |= {h - 1, h, h + 1}
    lows |= {0x3000, 0x6000, 0xA000, 0xC000, 0xE000, 0x9FFF, 0xBFFF}
    hi = np.arange(1 << 16, dtype=np.uint32) << np.uint32(16)
    lo = np.array(sorted(lows), np.uint32)
    structured = (hi[:, None] | lo[None, :]).ravel()
    rng = np.random.default_rng(seed)
    rand = rng.integers(0, 1 << 32, 1 << 25, dtype=np.uint64).astype(np.uint32)
    return np.concatenate([structured, rand])


def _chunks():
    if EXHAUSTIVE:
        step = 1 << 27
        for start in range(0, 1 << 32, step):
            yield np.arange(start, start + step, dtype=np.uint64).astype(np.uint32)
    else:
        yield _structured_f32_patterns(11)


def test_f32_to_bf16_all_rounding_classes(oracle_lib):
    """Against torch's CPU round-to-nearest-even: every upper half with every
    rounding class of the lower half (all 2^32 patterns with TS_EXHAUSTIVE=1)."""
    import torch

    for bits in _chunks():
        x = bits.view(np.float32)
        got = oracle_lib.f32_to_bf16(x)
        ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        nan = np.isnan(x)
        assert np.array_equal(got[~nan], ref[~nan])
        g = got[nan]
        assert np.all((g & 0x7F80) == 0x7F80) and np.all(g & 0x007F)  # NaN stays NaN
        assert np.array_equal(g & 0x8000, ((bits[nan] >> 16) & 0x8000).astype(np.uint16))


def test_f32_to_f16_all_rounding_classes(oracle_lib):
    """Against numpy's round-to-nearest-even (subnormals, overflow, ties)."""
    for bits in _chunks():
        x = bits.view(np.float32)
        got = oracle_lib.f32_to_f16(x)
        with np.errstate(over="ignore", invalid="ignore"):
            ref = x.astype(np.float16).view(np.uint16)
        nan = np.isnan(x)
        assert np.array_equal(got[~nan], ref[~nan])
        g = got[nan]
        assert np.all((g & 0x7C00) == 0x7C00) and np.all(g & 0x03FF)


def test_widening_exhaustive(oracle_lib):
    import torch

    h = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    f16 = oracle_lib.f16_to_f32(h)
    ref16 = h.view(np.float16).astype(np.float32)
    bf = oracle_lib.bf16_to_f32(h)
    refbf = torch.from_numpy(h.view(np.int16).copy()).view(torch.bfloat16).float().numpy()
    for got, ref in ((f16, ref16), (bf, refbf)):
        nan = np.isnan(ref)
        assert np.array_equal(np.isnan(got), nan)
        assert np.array_equal(got[~nan].view(np.uint32), ref[~nan].view(np.uint32))


def test_converter_edge_cases(oracle_lib):
    o = oracle_lib
    L = o.lib()
    # ties to even at the binary16 subnormal boundary and at 1.0
    assert L.oracle_f32_to_f16(2.0 ** -25) == 0x0000          # tie -> even (0)
    assert L.oracle_f32_to_f16(np.float32(2.0 ** -25 * 1.0000001)) == 0x0001
    assert L.oracle_f32_to_f16(3 * 2.0 ** -25) == 0x0002      # tie -> even (2)
    assert L.oracle_f32_to_f16(65504.0) == 0x7BFF
    assert L.oracle_f32_to_f16(65520.0) == 0x7C00             # tie above max -> inf
    assert L.oracle_f32_to_f16(np.float32(65519.99)) == 0x7BFF
    assert L.oracle_f32_to_f16(-0.0) == 0x8000
    assert L.oracle_f32_to_bf16(1.0 + 2.0 ** -8) == 0x3F80    # tie -> even
    assert L.oracle_f32_to_bf16(1.0 + 3 * 2.0 ** -8) == 0x3F82
    assert L.oracle_f32_to_bf16(-0.0) == 0x8000
    assert L.oracle_f32_to_bf16(float("inf")) == 0x7F80


# ------------------------------------------------------------- validation sums
def test_checksum_against_fsum(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, 10001)
    expected = 0.25
    x[::97] = expected
    cs = o.checksum(o.F64, x, expected)
    exact_sum = math.fsum(x.tolist())
    bound = x.size * 2.0 ** -53 * float(np.sum(np.abs(x)))
    assert abs(cs.sum - exact_sum) <= bound
    dev = np.abs(x - expected)
    assert abs(cs.abs_dev_sum - math.fsum(dev.tolist())) <= x.size * 2.0 ** -53 * float(dev.sum())
    assert cs.max_abs_dev == float(dev.max())
    assert cs.mismatches == int(np.count_nonzero(x != expected))


def test_checksum_nan_and_signed_zero(oracle_lib):
    o = oracle_lib
    x = np.array([0.0, -0.0, np.nan, 1.0], np.float64)
    cs = o.checksum(o.F64, x, 0.0)
    assert cs.mismatches == 3          # -0 differs from +0 in bits; NaN; 1.0
    assert cs.max_abs_dev == 1.0       # NaN deviation ignored as by fmax
    cs = o.checksum(o.F64, np.array([np.nan, np.nan]), float("nan"))
    assert cs.mismatches == 0
    assert o.checksum(o.F64, np.zeros(0), 1.0).sum == 0.0


def test_mismatch_count(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, 5000)
    ref = x.copy()
    idx = rng.choice(5000, 17, replace=False)
    ref[idx] = np.nextafter(ref[idx], np.inf)
    assert o.mismatch_count(o.F64, x, ref) == 17
    x16 = tsgen.narrow(x, "bf16")
    r16 = x16.copy()
    r16[idx[:5]] ^= np.uint16(1)
    assert o.mismatch_count(o.BF16, x16, r16) == 5


# ------------------------------------------------------------------ timed mode
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_timed_mode_closed_form(oracle_lib, threads):
    secs, fin, used = oracle_lib.stream_timed_f64(100003, 4, threads)
    assert used == threads
    assert secs.shape == (4, 4) and np.all(secs > 0)
    exp = (15.0 ** 4, 3 * 15.0 ** 3, 4 * 15.0 ** 3)
    assert tuple(fin[:3]) == exp and tuple(fin[3:]) == exp


def test_timed_mode_rejects_bad_args(oracle_lib):
    with pytest.raises(RuntimeError):
        oracle_lib.stream_timed_f64(0, 1, 1)
