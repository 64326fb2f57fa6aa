"""Exact rational reference arithmetic used to pin the oracle.

Each IEEE-754 operation is evaluated exactly with ``fractions.Fraction`` and
rounded once, to nearest with ties to even, to a binary format given by its
precision p (significand bits, hidden bit included) and exponent range.  Zero
results get their sign from the IEEE-754 rules, which a Fraction cannot carry.
This file shares no code with the oracle or the GPU library.
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction

# (precision bits, minimum normal exponent, maximum exponent)
FORMATS = {
    "f64": (53, -1022, 1023),
    "f32": (24, -126, 127),
    "bf16": (8, -126, 127),
    "f16": (11, -14, 15),
}

INF = float("inf")


def round_fraction(v: Fraction, fmt: str) -> float:
    """Round the exact value v to format fmt (RNE, overflow to infinity).

    Returns a Python float holding the rounded value exactly (every value of
    these formats is a binary64 value).  Zero comes back as +0.0; callers fix
    its sign."""
    p, emin, emax = FORMATS[fmt]
    if v == 0:
        return 0.0
    neg = v < 0
    v = -v if neg else v
    e = v.numerator.bit_length() - v.denominator.bit_length()
    # settle e so that 2^e <= v < 2^(e+1)
    while Fraction(2) ** e > v:
        e -= 1
    while Fraction(2) ** (e + 1) <= v:
        e += 1
    e = max(e, emin)  # below the normal range the quantum stays 2^(emin-p+1)
    quantum = Fraction(2) ** (e - p + 1)
    m = v / quantum
    mi = m.numerator // m.denominator
    rem = m - mi
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and mi % 2 == 1):
        mi += 1
    r = mi * quantum
    if r >= Fraction(2) ** (emax + 1):
        return -INF if neg else INF
    f = float(r)  # exact: r is representable in binary64
    return -f if neg else f


def _signbit(x: float) -> bool:
    return math.copysign(1.0, x) < 0


def _finite_or_none(*xs):
    return all(math.isfinite(x) for x in xs)


def mul(a: float, b: float, fmt: str) -> float:
    if not _finite_or_none(a, b):
        return a * b  # IEEE special cases are the same in every format here
    exact = Fraction(a) * Fraction(b)
    r = round_fraction(exact, fmt)
    if r == 0:
        return math.copysign(0.0, -1.0 if _signbit(a) != _signbit(b) else 1.0)
    return r


def add(a: float, b: float, fmt: str) -> float:
    if not _finite_or_none(a, b):
        return a + b
    exact = Fraction(a) + Fraction(b)
    r = round_fraction(exact, fmt)
    if r == 0:
        if exact == 0:
            both_neg = _signbit(a) and _signbit(b)
            return -0.0 if both_neg else 0.0
        return math.copysign(0.0, -1.0 if exact < 0 else 1.0)
    return r


def fma(q: float, y: float, x: float, fmt: str) -> float:
    """q*y + x with one rounding."""
    if not _finite_or_none(q, y, x):
        # With an infinite or NaN operand the result is infinite or NaN and
        # no rounding is involved; IEEE float arithmetic gives it directly
        # (a finite q*y cannot overflow binary64 for the formats used here).
        return q * y + x
    prod = Fraction(q) * Fraction(y)
    exact = prod + Fraction(x)
    r = round_fraction(exact, fmt)
    if r == 0:
        if exact == 0:
            prod_neg = _signbit(q) != _signbit(y)
            if prod == 0 and x == 0:
                return -0.0 if (prod_neg and _signbit(x)) else 0.0
            return 0.0
        return math.copysign(0.0, -1.0 if exact < 0 else 1.0)
    return r


def narrow(x: float, fmt: str) -> float:
    """Round a binary64 value (already exact) into fmt."""
    if not math.isfinite(x):
        return x
    r = round_fraction(Fraction(x), fmt)
    if r == 0:
        return math.copysign(0.0, -1.0 if _signbit(x) else 1.0)
    return r


def f64_bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def stream_scalar(a: float, b: float, c: float, q: float, iterations: int, fmt: str = "f64",
                  fused: bool = True):
    """The benchmark iteration (copy, scale, add, triad) on one element, every
    operation rounded once into fmt.  fused=False rounds the triad's product
    and sum separately (the unfused reading), to show the two differ."""
    for _ in range(iterations):
        c = a
        b = mul(q, c, fmt)
        c = add(a, b, fmt)
        if fused:
            a = fma(q, c, b, fmt)
        else:
            a = add(b, mul(q, c, fmt), fmt)
    return a, b, c
