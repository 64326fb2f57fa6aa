"""CPU oracle for the STREAM hot path -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and
shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C loops compiled by gcc with
``-ffp-contract=off``); this module builds that file into ``liboracle.so`` and
exposes numpy-friendly wrappers.  What each function computes, and which
passage of the paper it follows, is documented in ``oracle.h``: the four maps
of the generic STREAM benchmark (Section 5, Listing 4) -- copy c = a,
scale b = q*c, add c = a + b, triad a = b + q*c as one fused multiply-add.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
COPY, SCALE, ADD, TRIAD = 0, 1, 2, 3
OPS = {"copy": COPY, "scale": SCALE, "add": ADD, "triad": TRIAD}

# Storage numpy dtype per oracle dtype (16-bit formats travel as raw uint16).
_NP = {F64: np.float64, F32: np.float32, BF16: np.uint16, F16: np.uint16}
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU, no HIP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = [
        "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
        "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class Checksum(ctypes.Structure):
    _fields_ = [
        ("sum", ctypes.c_double),
        ("abs_dev_sum", ctypes.c_double),
        ("max_abs_dev", ctypes.c_double),
        ("mismatches", ctypes.c_uint64),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liboracle.so, building it first if it is missing or stale."""
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P, S, D, I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double, ctypes.c_int
        for name, args in {
            "oracle_copy_f64": [P, P, S],
            "oracle_scale_f64": [P, P, S, D],
            "oracle_add_f64": [P, P, P, S],
            "oracle_triad_f64": [P, P, P, S, D],
            "oracle_stream_iteration_f64": [P, P, P, S, D],
            "oracle_stream_run_f64": [P, P, P, S, D, I],
            "oracle_stream_run_copyb_f64": [P, P, P, S, D, I],
            "oracle_f32_to_bf16_array": [P, P, S],
            "oracle_f32_to_f16_array": [P, P, S],
            "oracle_bf16_to_f32_array": [P, P, S],
            "oracle_f16_to_f32_array": [P, P, S],
        }.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, None
        for name, args in {
            "oracle_op": [I, I, P, P, P, S, D],
            "oracle_stream_run": [I, P, P, P, S, D, I],
            "oracle_checksum_array": [I, P, S, D, ctypes.POINTER(Checksum)],
            "oracle_mismatch_count": [I, P, P, S, ctypes.POINTER(ctypes.c_uint64)],
            "oracle_stream_timed_f64": [S, I, I, D, P, P, ctypes.POINTER(ctypes.c_int)],
        }.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, ctypes.c_int
        L.oracle_f32_to_bf16.argtypes, L.oracle_f32_to_bf16.restype = [ctypes.c_float], ctypes.c_uint16
        L.oracle_f32_to_f16.argtypes, L.oracle_f32_to_f16.restype = [ctypes.c_float], ctypes.c_uint16
        L.oracle_bf16_to_f32.argtypes, L.oracle_bf16_to_f32.restype = [ctypes.c_uint16], ctypes.c_float
        L.oracle_f16_to_f32.argtypes, L.oracle_f16_to_f32.restype = [ctypes.c_uint16], ctypes.c_float
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags.c_contiguous
    return a.ctypes.data


def _check(a: np.ndarray, dtype: int, n: int, name: str) -> None:
    if a.dtype != _NP[dtype] or a.ndim != 1 or a.shape[0] < n or not a.flags.c_contiguous:
        raise ValueError(f"{name}: need a contiguous 1-D {np.dtype(_NP[dtype])} array of >= {n} elements")


def op(dtype: int, which: int, x: np.ndarray, y: np.ndarray | None, dst: np.ndarray, q: float = 3.0,
       n: int | None = None) -> np.ndarray:
    """One map of Listing 4 (COPY/SCALE/ADD/TRIAD) over storage arrays; writes dst."""
    n = x.shape[0] if n is None else n
    _check(x, dtype, n, "x")
    _check(dst, dtype, n, "dst")
    if which in (ADD, TRIAD):
        _check(y, dtype, n, "y")
    rc = lib().oracle_op(dtype, which, _ptr(x), _ptr(y) if which in (ADD, TRIAD) else None, _ptr(dst), n, q)
    if rc != 0:
        raise ValueError("oracle_op: bad dtype or op")
    return dst


def stream_run(dtype: int, a: np.ndarray, b: np.ndarray, c: np.ndarray, q: float = 3.0,
               iterations: int = 1) -> None:
    """``iterations`` benchmark iterations in listing order, in place."""
    n = a.shape[0]
    for arr, nm in ((a, "a"), (b, "b"), (c, "c")):
        _check(arr, dtype, n, nm)
    if dtype == F64:
        lib().oracle_stream_run_f64(_ptr(a), _ptr(b), _ptr(c), n, q, iterations)
    else:
        lib().oracle_stream_run(dtype, _ptr(a), _ptr(b), _ptr(c), n, q, iterations)


def stream_run_copyb_f64(a: np.ndarray, b: np.ndarray, c: np.ndarray, q: float = 3.0,
                         iterations: int = 1) -> None:
    """The variant with copy a <- b (scale, add, triad as listed), in place."""
    n = a.shape[0]
    for arr, nm in ((a, "a"), (b, "b"), (c, "c")):
        _check(arr, F64, n, nm)
    lib().oracle_stream_run_copyb_f64(_ptr(a), _ptr(b), _ptr(c), n, q, iterations)


def stream_scalar_f64(a0: float, b0: float, c0: float, q: float, iterations: int):
    """The iteration applied to one element (every element evolves alone)."""
    a = np.array([a0], np.float64)
    b = np.array([b0], np.float64)
    c = np.array([c0], np.float64)
    lib().oracle_stream_run_f64(_ptr(a), _ptr(b), _ptr(c), 1, q, iterations)
    return float(a[0]), float(b[0]), float(c[0])


def stream_elements_f64(a0: np.ndarray, b0: np.ndarray, c0: np.ndarray, q, iterations: int):
    """Iterate a set of independent elements (e.g. sampled indices of a big
    array, or one element of each batched instance with its own q)."""
    a = np.ascontiguousarray(a0, np.float64).copy()
    b = np.ascontiguousarray(b0, np.float64).copy()
    c = np.ascontiguousarray(c0, np.float64).copy()
    qs = np.broadcast_to(np.asarray(q, np.float64), a.shape)
    if np.all(qs == qs.flat[0]) if qs.size else True:
        if a.size:
            lib().oracle_stream_run_f64(_ptr(a), _ptr(b), _ptr(c), a.size, float(qs.flat[0]), iterations)
        return a, b, c
    for qv in np.unique(qs):
        idx = np.nonzero(qs == qv)[0]
        sa, sb, sc = a[idx].copy(), b[idx].copy(), c[idx].copy()
        lib().oracle_stream_run_f64(_ptr(sa), _ptr(sb), _ptr(sc), idx.size, float(qv), iterations)
        a[idx], b[idx], c[idx] = sa, sb, sc
    return a, b, c


def f32_to_bf16(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty(x.shape, np.uint16)
    lib().oracle_f32_to_bf16_array(_ptr(x), _ptr(out), x.size)
    return out


def f32_to_f16(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty(x.shape, np.uint16)
    lib().oracle_f32_to_f16_array(_ptr(x), _ptr(out), x.size)
    return out


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    h = np.ascontiguousarray(h, np.uint16)
    out = np.empty(h.shape, np.float32)
    lib().oracle_bf16_to_f32_array(_ptr(h), _ptr(out), h.size)
    return out


def f16_to_f32(h: np.ndarray) -> np.ndarray:
    h = np.ascontiguousarray(h, np.uint16)
    out = np.empty(h.shape, np.float32)
    lib().oracle_f16_to_f32_array(_ptr(h), _ptr(out), h.size)
    return out


def widen_f64(dtype: int, x: np.ndarray) -> np.ndarray:
    """Exact binary64 value of each stored element."""
    if dtype == F64:
        return x.astype(np.float64)
    if dtype == F32:
        return x.astype(np.float64)
    if dtype == BF16:
        return bf16_to_f32(x).astype(np.float64)
    return f16_to_f32(x).astype(np.float64)


def checksum(dtype: int, x: np.ndarray, expected: float, n: int | None = None) -> Checksum:
    n = x.shape[0] if n is None else n
    _check(x, dtype, n, "x")
    out = Checksum()
    if lib().oracle_checksum_array(dtype, _ptr(x), n, expected, ctypes.byref(out)) != 0:
        raise ValueError("oracle_checksum_array failed")
    return out


def mismatch_count(dtype: int, x: np.ndarray, ref: np.ndarray, n: int | None = None) -> int:
    n = x.shape[0] if n is None else n
    _check(x, dtype, n, "x")
    _check(ref, dtype, n, "ref")
    out = ctypes.c_uint64()
    if lib().oracle_mismatch_count(dtype, _ptr(x), _ptr(ref), n, ctypes.byref(out)) != 0:
        raise ValueError("oracle_mismatch_count failed")
    return int(out.value)


def stream_timed_f64(n: int, iterations: int, threads: int, q: float = 3.0):
    """Timed host run (block-partitioned pinned threads, first touch).

    Returns (op_seconds[iterations, 4], final_abc[6], threads_used)."""
    secs = np.zeros(4 * max(iterations, 1), np.float64)
    fin = np.zeros(6, np.float64)
    used = ctypes.c_int(0)
    rc = lib().oracle_stream_timed_f64(n, iterations, threads, q, _ptr(secs), _ptr(fin), ctypes.byref(used))
    if rc != 0:
        raise RuntimeError(f"oracle_stream_timed_f64 failed ({rc})")
    return secs[: 4 * iterations].reshape(iterations, 4), fin, used.value
