"""Seeded synthetic inputs for the STREAM workloads.

This module only *draws inputs*; it holds none of the benchmark's arithmetic.
The GPU library's fill kernel implements the same counter-based generator
from its published definition, independently, so that large arrays can be
constructed in place on the device; tests compare the two bit for bit.

Generator (counter-based, so any element can be recomputed alone):

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014; the finaliser with constants 0xbf58476d1ce4e5b9 and
  0x94d049bb133111eb and shifts 30/27/31, golden gamma 0x9e3779b97f4a7c15).
  Element j of stream s under seed k is the (j+1)-th output of a SplitMix64
  whose initial state is ``k XOR (s << 48)``:
  ``h = mix((k ^ (s << 48)) + (j + 1) * gamma)`` (mod 2^64).
* ``uniform_pm1``: ``(h >> 11) * 2^-52 - 1``, an exact binary64 value in
  [-1, 1) on a grid of 2^-52.
* ``uniform01``: ``(h >> 11) * 2^-53`` in [0, 1).
* Storage narrowing: binary64 -> binary32 by round-to-nearest-even; bfloat16
  and binary16 inputs are then narrowed from that binary32 value by
  round-to-nearest-even (i.e. inputs are defined as RNE_D(RNE_f32(u))).

Streams: a = 0, b = 1, c = 2, batched lengths = 3, batched q = 4; batched
instance i draws its a, b, c from streams 16 + 3i + {0, 1, 2}.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_A, STREAM_B, STREAM_C, STREAM_LEN, STREAM_Q = 0, 1, 2, 3, 4


def instance_stream(i: int, which: int) -> int:
    """Stream id of batched instance i, array which (0 = a, 1 = b, 2 = c)."""
    return 16 + 3 * int(i) + int(which)


def splitmix64_mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def raw(seed: int, stream: int, idx) -> np.ndarray:
    """64-bit outputs for element indices ``idx`` (array-like of int)."""
    idx = np.asarray(idx, np.uint64)
    base = np.uint64((int(seed) ^ (int(stream) << 48)) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        z = base + (idx + np.uint64(1)) * GAMMA
    return splitmix64_mix(z)


def uniform_pm1(seed: int, stream: int, idx) -> np.ndarray:
    h = raw(seed, stream, idx)
    return (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def uniform01(seed: int, stream: int, idx) -> np.ndarray:
    h = raw(seed, stream, idx)
    return (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def _f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    import torch  # torch's CPU conversion is round-to-nearest-even

    t = torch.from_numpy(np.ascontiguousarray(x32, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16).copy()


def narrow(x64: np.ndarray, dtype: str) -> np.ndarray:
    """Storage array for dtype in {'f64','f32','bf16','f16'}; 16-bit formats
    are returned as raw uint16 bit patterns."""
    x64 = np.asarray(x64, np.float64)
    if dtype == "f64":
        return x64.copy()
    with np.errstate(over="ignore"):  # overflow rounds to infinity, as IEEE 754 defines
        x32 = x64.astype(np.float32)
        if dtype == "f32":
            return x32
        if dtype == "f16":
            return x32.astype(np.float16).view(np.uint16)
    if dtype == "bf16":
        return _f32_to_bf16_bits(x32)
    raise ValueError(dtype)


def uniform_range(seed: int, stream: int, idx, lo: float, hi: float) -> np.ndarray:
    """lo + (hi - lo) * u01, the difference, the product and the sum each
    rounded once in binary64 (numpy does not contract)."""
    w = np.float64(hi) - np.float64(lo)
    return np.float64(lo) + w * uniform01(seed, stream, idx)


def uniform_array(seed: int, stream: int, n: int, dtype: str = "f64", start: int = 0,
                  lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Elements start..start+n-1 of a seeded uniform array over [lo, hi)
    (the default [-1, 1) draws exact multiples of 2^-52)."""
    idx = np.arange(start, start + n, dtype=np.uint64)
    if (lo, hi) == (-1.0, 1.0):
        return narrow(uniform_pm1(seed, stream, idx), dtype)
    return narrow(uniform_range(seed, stream, idx, lo, hi), dtype)


def batched_lengths(seed: int, count: int, lo_exp: float = 3.0, span_exp: float = 4.0) -> np.ndarray:
    """Log-uniform instance lengths floor(10^(lo + span*u)), u in [0,1)."""
    u = uniform01(seed, STREAM_LEN, np.arange(count, dtype=np.uint64))
    return np.floor(np.power(10.0, lo_exp + span_exp * u)).astype(np.uint64)


def batched_scalars(seed: int, count: int, lo: float = 0.5, hi: float = 4.0) -> np.ndarray:
    """Per-instance scalars q_i = lo + (hi - lo) * u."""
    u = uniform01(seed, STREAM_Q, np.arange(count, dtype=np.uint64))
    return lo + (hi - lo) * u
