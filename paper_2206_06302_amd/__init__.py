"""Python binding of libtstream: STREAM on placed arrays and execution targets.

Mirrors the usage pattern of the paper's hello-world example (Section 3.4,
Listing 3): make a target, place arrays on it, run algorithms on it.

    import torch, paper_2206_06302_amd as ts
    tgt = ts.Target(0, torch.cuda.Stream())          # device + stream (Section 4.2)
    a = ts.Array.wrap(tgt, torch.empty(n, dtype=torch.float64, device="cuda"))
    ...
    ts.copy(tgt, a, c); ts.scale(tgt, c, b, 3.0)    # Listing 4, in order
    ts.add(tgt, a, b, c); ts.triad(tgt, b, c, a, 3.0)

Every call is argument marshalling around one C-ABI function; every step of
the STREAM path runs in the library's HIP kernels.  torch supplies device
memory and streams only.  Importing fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os
import warnings

import numpy as np
import torch  # must load first: libtstream then binds to torch's HIP runtime

from . import _lib
from ._lib import BatchDescC, ChecksumOut, DeviceInfo, KernelCfg, ProbeCfg

lib = _lib.load()

_runtimes = _lib.hip_runtimes_loaded()
if len(_runtimes) > 1:
    raise ImportError("two HIP runtimes are loaded in this process (%s); streams would not be "
                      "shared between torch and libtstream" % ", ".join(_runtimes))

DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "u8": 4}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}
TORCH_DTYPES = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16,
                "u8": torch.uint8}
_FROM_TORCH = {v: k for k, v in TORCH_DTYPES.items()}
ELEM_SIZE = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "u8": 1}
NP_STORAGE = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16, "f16": np.uint16, "u8": np.uint8}
OPS = {"copy": 0, "scale": 1, "add": 2, "triad": 3}
ALIGN_16, ALIGN_SHARED, ALIGN_MIXED = 0, 1, 2
# STREAM bytes per element: copy/scale move two arrays, add/triad three.
ARRAYS_MOVED = {"copy": 2, "scale": 2, "add": 3, "triad": 3}
HIP_STREAM_LEGACY = 1  # HIP's handle of a device's legacy default stream (hipStreamLegacy)

DEFAULT_TUNE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune", "gfx950.json")


class TSError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.message = message
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")


def last_error() -> str:
    m = lib.ts_last_error()
    return m.decode() if m else ""


def _check(rc: int) -> int:
    if rc < 0:
        raise TSError(rc, last_error())
    return rc


def _dt(dtype) -> int:
    if isinstance(dtype, torch.dtype):
        dtype = _FROM_TORCH[dtype]
    if isinstance(dtype, str):
        return DTYPES[dtype]
    return int(dtype)


def _op(op) -> int:
    return OPS[op] if isinstance(op, str) else int(op)


def host_numa_domains() -> list[list[int]]:
    """CPU ids of each NUMA domain the process may run on."""
    cnt = ctypes.c_int()
    _check(lib.ts_host_numa_domains(ctypes.byref(cnt)))
    out = []
    for d in range(cnt.value):
        n = ctypes.c_int()
        _check(lib.ts_host_domain_cpus(d, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_int * max(1, n.value))()
        _check(lib.ts_host_domain_cpus(d, buf, n.value, ctypes.byref(n)))
        out.append(list(buf[:n.value]))
    return out


def version() -> tuple[int, int]:
    ma, mi = ctypes.c_int(), ctypes.c_int()
    _check(lib.ts_version(ctypes.byref(ma), ctypes.byref(mi)))
    return ma.value, mi.value


# ---------------------------------------------------------------------------
# Targets (Section 3.1; GPU target = device + stream, Section 4.2)
# ---------------------------------------------------------------------------
class Target:
    """A device plus the stream its work is ordered on.

    ``stream`` may be a torch stream, a raw hipStream_t (int; 0 is the
    device's default stream), ``None`` for torch's current stream of the
    device, or ``"own"`` for a non-blocking stream the library creates."""

    def __init__(self, device: int = 0, stream=None):
        self._torch_stream = None
        h = ctypes.c_void_p()
        if isinstance(stream, str):
            if stream != "own":
                raise ValueError("stream must be a torch stream, an int handle, None or 'own'")
            _check(lib.ts_target_create_owned(int(device), ctypes.byref(h)))
        else:
            if stream is None:
                stream = torch.cuda.current_stream(device)
            if isinstance(stream, torch.cuda.Stream):
                self._torch_stream = stream
                raw = stream.cuda_stream
            else:
                raw = int(stream)
            # torch's default stream is the legacy null stream: pass HIP's
            # handle for it (NULL would ask for a stream of the library's own)
            _check(lib.ts_target_create(int(device), ctypes.c_void_p(raw if raw else HIP_STREAM_LEGACY),
                                        ctypes.byref(h)))
        self.handle = h
        self.device = int(device)
        self._callbacks = []

    @classmethod
    def host(cls, cpus=None) -> "Target":
        """Host-CPU target: one pinned worker per CPU in `cpus` (default: every
        CPU the process may use, grouped by NUMA domain); arrays on it are
        divided into equal blocks over the workers (Section 4.1)."""
        self = cls.__new__(cls)
        self._torch_stream = None
        self._callbacks = []
        h = ctypes.c_void_p()
        if cpus:
            arr = (ctypes.c_int * len(cpus))(*[int(c) for c in cpus])
            _check(lib.ts_target_create_host(arr, len(cpus), ctypes.byref(h)))
        else:
            _check(lib.ts_target_create_host(None, 0, ctypes.byref(h)))
        self.handle = h
        self.device = -1
        return self

    def synchronize(self) -> None:
        _check(lib.ts_target_synchronize(self.handle))

    def info(self) -> dict:
        d = DeviceInfo()
        _check(lib.ts_target_info(self.handle, ctypes.byref(d)))
        out = {f: getattr(d, f) for f, _ in d._fields_}
        out["arch"] = d.arch.decode()
        out["name"] = d.name.decode()
        return out

    def stream_handle(self) -> int:
        p = ctypes.c_void_p()
        _check(lib.ts_target_stream(self.handle, ctypes.byref(p)))
        return p.value or 0

    def then(self, fn) -> None:
        """Run fn() on a runtime thread once all work enqueued so far is done."""
        def tramp(_user):
            fn()
        cb = _lib.CALLBACK(tramp)
        self._callbacks.append(cb)  # keep alive until the target goes away
        _check(lib.ts_target_then(self.handle, cb, None))

    def async_(self) -> "Future":
        """Future of all work enqueued so far (ready from a stream callback)."""
        h = ctypes.c_void_p()
        _check(lib.ts_target_async(self.handle, ctypes.byref(h)))
        return Future(h)

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.ts_target_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Arrays (Section 3.2)
# ---------------------------------------------------------------------------
class Array:
    """A contiguous 1-D array placed on a target's device."""

    def __init__(self, handle, target: Target, dtype: str, n: int, keep=None):
        self.handle = handle
        self.target = target
        self.dtype = dtype
        self.n = n
        self._keep = keep

    @classmethod
    def wrap(cls, target: Target, tensor: torch.Tensor, n: int | None = None) -> "Array":
        """Borrow a torch tensor's memory (the tensor is kept alive)."""
        if not tensor.is_cuda:
            raise TSError(-4, "tensor is not device memory")
        if not tensor.is_contiguous():
            raise TSError(-1, "tensor must be contiguous")
        dtype = _FROM_TORCH.get(tensor.dtype)
        if dtype is None:
            raise TSError(-3, f"unsupported tensor dtype {tensor.dtype}")
        n = tensor.numel() if n is None else int(n)
        h = ctypes.c_void_p()
        _check(lib.ts_array_wrap(target.handle, DTYPES[dtype], ctypes.c_void_p(tensor.data_ptr()), n,
                                 ctypes.byref(h)))
        return cls(h, target, dtype, n, keep=tensor)

    @classmethod
    def wrap_numpy(cls, target: Target, arr: np.ndarray) -> "Array":
        """Borrow a contiguous 1-D numpy array (host memory; host targets)."""
        names = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32", np.dtype(np.uint8): "u8"}
        dtype = names.get(arr.dtype)
        if dtype is None or arr.ndim != 1 or not arr.flags.c_contiguous:
            raise TSError(-3, "need a contiguous 1-D float64, float32 or uint8 array")
        h = ctypes.c_void_p()
        _check(lib.ts_array_wrap(target.handle, DTYPES[dtype], ctypes.c_void_p(arr.ctypes.data), arr.size,
                                 ctypes.byref(h)))
        return cls(h, target, dtype, arr.size, keep=arr)

    @classmethod
    def alloc(cls, target: Target, dtype: str, n: int, offset: int = 0) -> "Array":
        h = ctypes.c_void_p()
        _check(lib.ts_array_alloc(target.handle, _dt(dtype), int(n), int(offset), ctypes.byref(h)))
        return cls(h, target, dtype if isinstance(dtype, str) else DTYPE_NAMES[_dt(dtype)], int(n))

    def ptr(self) -> int:
        p = ctypes.c_void_p()
        _check(lib.ts_array_info(self.handle, ctypes.byref(p), None, None))
        return p.value or 0

    def fill(self, value: float) -> "Array":
        _check(lib.ts_fill(self.handle, float(value)))
        return self

    def fill_uniform(self, seed: int, stream_id: int, first_index: int = 0, lo: float = -1.0,
                     hi: float = 1.0) -> "Array":
        if (lo, hi) == (-1.0, 1.0):
            _check(lib.ts_fill_uniform(self.handle, int(seed), int(stream_id), int(first_index)))
        else:
            _check(lib.ts_fill_uniform_range(self.handle, int(seed), int(stream_id), int(first_index),
                                             float(lo), float(hi)))
        return self

    def copy_from_host(self, host: np.ndarray) -> None:
        host = np.ascontiguousarray(host, NP_STORAGE[self.dtype])
        _check(lib.ts_copy_from_host(self.handle, host.ctypes.data, host.size))
        self.target.synchronize()  # the host buffer may be released after return

    def to_host(self, n: int | None = None) -> np.ndarray:
        """Blocking device-to-host copy of the first n elements (storage bits
        for the 16-bit formats, as uint16)."""
        n = self.n if n is None else int(n)
        out = np.empty(n, NP_STORAGE[self.dtype])
        _check(lib.ts_copy_to_host(out.ctypes.data, self.handle, n))
        self.target.synchronize()
        return out

    def free(self) -> None:
        if self.handle:
            lib.ts_array_free(self.handle)
            self.handle = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Algorithms (Section 3.4; the maps of Listing 4)
# ---------------------------------------------------------------------------
def copy(target: Target, src: Array, dst: Array) -> None:
    """dst = src (Listing 4, Copy)."""
    _check(lib.ts_copy(target.handle, src.handle, dst.handle))


def scale(target: Target, src: Array, dst: Array, q: float) -> None:
    """dst = q * src (Listing 4, Scale)."""
    _check(lib.ts_scale(target.handle, src.handle, dst.handle, float(q)))


def add(target: Target, x: Array, y: Array, dst: Array) -> None:
    """dst = x + y (Listing 4, Add)."""
    _check(lib.ts_add(target.handle, x.handle, y.handle, dst.handle))


def triad(target: Target, x: Array, y: Array, dst: Array, q: float) -> None:
    """dst = x + q * y with one rounding (Listing 4, Triad: a = b + q*c is
    triad(t, b, c, a, q))."""
    _check(lib.ts_triad(target.handle, x.handle, y.handle, dst.handle, float(q)))


ORDERS = ("listing", "copy_b")


def stream_iteration(target: Target, a: Array, b: Array, c: Array, q: float = 3.0,
                     order: str = "listing") -> None:
    """One iteration of Listing 4: c = a; b = q*c; c = a + b; a = b + q*c.
    order="copy_b" runs the variant whose copy is a = b (the direction some
    summaries of STREAM write), the other maps unchanged, as four calls."""
    if order == "listing":
        _check(lib.ts_stream_iteration(target.handle, a.handle, b.handle, c.handle, float(q)))
    elif order == "copy_b":
        copy(target, b, a)
        scale(target, c, b, q)
        add(target, a, b, c)
        triad(target, b, c, a, q)
    else:
        raise ValueError(f"order must be one of {ORDERS}")


def run_op(target: Target, op, x: Array, y: Array | None, dst: Array, q: float = 3.0) -> None:
    op = _op(op)
    if op == 0:
        copy(target, x, dst)
    elif op == 1:
        scale(target, x, dst, q)
    elif op == 2:
        add(target, x, y, dst)
    else:
        triad(target, x, y, dst, q)


def checksum(target: Target, x: Array, expected: float) -> dict:
    out = ChecksumOut()
    _check(lib.ts_checksum(target.handle, x.handle, float(expected), ctypes.byref(out)))
    return {"sum": out.sum, "abs_dev_sum": out.abs_dev_sum, "max_abs_dev": out.max_abs_dev,
            "mismatches": int(out.mismatches)}


def checksum_noalloc(target: Target, x: Array, expected: float, dev_out: int) -> None:
    """ts_checksum_noalloc: enqueue the checksum of x with its result stored
    at the device address dev_out (32 bytes: sum, abs_dev_sum, max_abs_dev as
    binary64, then mismatches as uint64).  Does not wait."""
    _check(lib.ts_checksum_noalloc(target.handle, x.handle, float(expected), ctypes.c_void_p(int(dev_out))))


def mismatch_count(target: Target, x: Array, ref: Array) -> int:
    out = ctypes.c_uint64()
    _check(lib.ts_mismatch_count(target.handle, x.handle, ref.handle, ctypes.byref(out)))
    return int(out.value)


def time_op(target: Target, op, x: Array, y: Array | None, dst: Array, q: float = 3.0,
            reps: int = 10) -> float:
    """Milliseconds for `reps` back-to-back launches (event-timed, blocking)."""
    ms = ctypes.c_float()
    _check(lib.ts_time_op(target.handle, _op(op), x.handle, y.handle if y is not None else None,
                          dst.handle, float(q), int(reps), ctypes.byref(ms)))
    return float(ms.value)


def probe_bandwidth(target: Target, cfg: dict, x: Array | None, y: Array | None, dst: Array, nbytes: int,
                    mark: int = 0x5A5A5A5A) -> None:
    """One launch of the memory-system probe (ts_probe_bandwidth): cfg keys
    reads, writes, block, unroll, nt_load, nt_store, wave_contiguous,
    lds_bytes.  Asynchronous on the target's stream."""
    c = ProbeCfg.from_dict(cfg)
    _check(lib.ts_probe_bandwidth(target.handle, ctypes.byref(c), x.handle if x is not None else None,
                                  y.handle if y is not None else None, dst.handle, int(nbytes),
                                  int(mark) & 0xFFFFFFFF))


# ---------------------------------------------------------------------------
# Tuning
# ---------------------------------------------------------------------------
def get_kernel_cfg(op, dtype, n: int, align_class: int = ALIGN_16, batched: bool = False) -> dict:
    c = KernelCfg()
    _check(lib.ts_get_kernel_cfg(_op(op), _dt(dtype), int(n), int(align_class), int(bool(batched)),
                                 ctypes.byref(c)))
    return c.as_dict()


def set_kernel_cfg(op, dtype, cfg: dict | None, batched: bool = False) -> None:
    c = KernelCfg.from_dict(cfg) if cfg is not None else None
    _check(lib.ts_set_kernel_cfg(_op(op), _dt(dtype), int(bool(batched)),
                                 ctypes.byref(c) if c is not None else None))


def candidates(batched: bool = False) -> list[dict]:
    n = ctypes.c_size_t()
    _check(lib.ts_autotune_candidates(int(bool(batched)), None, 0, ctypes.byref(n)))
    arr = (KernelCfg * n.value)()
    _check(lib.ts_autotune_candidates(int(bool(batched)), arr, n.value, ctypes.byref(n)))
    return [c.as_dict() for c in arr]


def autotune(target: Target, op, dtype, n: int, offset: int = 0, reps: int = 5) -> tuple[dict, float]:
    c = KernelCfg()
    bps = ctypes.c_double()
    _check(lib.ts_autotune(target.handle, _op(op), _dt(dtype), int(n), int(offset), int(reps),
                           ctypes.byref(c), ctypes.byref(bps)))
    return c.as_dict(), bps.value


def autotune_batch(target: Target, batch: "Batch", op, reps: int = 3) -> tuple[dict, float]:
    c = KernelCfg()
    bps = ctypes.c_double()
    _check(lib.ts_autotune_batch(target.handle, batch.handle, _op(op), int(reps), ctypes.byref(c),
                                 ctypes.byref(bps)))
    return c.as_dict(), bps.value


def tune_cache_load(path: str) -> None:
    _check(lib.ts_tune_cache_load(os.fsencode(path)))


def tune_cache_save(path: str) -> None:
    _check(lib.ts_tune_cache_save(os.fsencode(path)))


def tune_cache_clear() -> None:
    _check(lib.ts_tune_cache_clear())


def load_default_tuning() -> bool:
    """Load the committed gfx950 tuning table if present (TS_TUNE_CACHE, when
    set, is loaded by the library itself at the first target)."""
    if os.path.exists(DEFAULT_TUNE_FILE):
        try:
            tune_cache_load(DEFAULT_TUNE_FILE)
            return True
        except TSError as e:
            warnings.warn(f"ignoring tuning table: {e}")
    return False


# ---------------------------------------------------------------------------
# Batched ragged instances
# ---------------------------------------------------------------------------
class Batch:
    """Ragged instances {a_i, b_i, c_i, len_i, q_i}; one launch per map."""

    def __init__(self, target: Target, dtype, descs, keep=None):
        arr = (BatchDescC * len(descs))()
        for i, (a, b, c, n, q) in enumerate(descs):
            arr[i].a, arr[i].b, arr[i].c, arr[i].len, arr[i].q = a, b, c, int(n), float(q)
        h = ctypes.c_void_p()
        _check(lib.ts_batch_create(target.handle, _dt(dtype), arr, len(descs), ctypes.byref(h)))
        self.handle = h
        self.target = target
        self.dtype = dtype if isinstance(dtype, str) else DTYPE_NAMES[_dt(dtype)]
        self.count = len(descs)
        self._keep = keep

    def info(self) -> dict:
        cnt, tot, tiles, te = ctypes.c_size_t(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int64()
        _check(lib.ts_batch_info(self.handle, ctypes.byref(cnt), ctypes.byref(tot), ctypes.byref(tiles),
                                 ctypes.byref(te)))
        return {"count": cnt.value, "total_elems": tot.value, "tiles": tiles.value, "tile_elems": te.value}

    def set_tile(self, tile_elems: int) -> None:
        _check(lib.ts_batch_set_tile(self.handle, int(tile_elems)))

    def op(self, target: Target, op) -> None:
        _check(lib.ts_batch_op(target.handle, self.handle, _op(op)))

    def op_plain(self, target: Target, op) -> None:
        _check(lib.ts_batch_op_plain(target.handle, self.handle, _op(op)))

    def fill(self, target: Target, which: int, value: float) -> None:
        _check(lib.ts_batch_fill(target.handle, self.handle, int(which), float(value)))

    def fill_uniform(self, target: Target, which: int, seed: int) -> None:
        _check(lib.ts_batch_fill_uniform(target.handle, self.handle, int(which), int(seed)))

    def mismatch_count(self, target: Target, which: int, expected) -> np.ndarray:
        exp = np.ascontiguousarray(expected, np.float64)
        if exp.size != self.count:
            raise TSError(-2, "one expected value per instance is required")
        counts = np.zeros(self.count, np.uint64)
        _check(lib.ts_batch_mismatch_count(target.handle, self.handle, int(which), exp.ctypes.data,
                                           counts.ctypes.data))
        return counts

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.ts_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """An instantiated HIP graph of STREAM launches."""

    def __init__(self, handle, keep=None):
        self.handle = handle
        self._keep = keep

    @classmethod
    def capture_stream_iteration(cls, target: Target, batch: Batch, iterations: int = 1) -> "Graph":
        """`iterations` consecutive batched iterations (4 nodes each)."""
        h = ctypes.c_void_p()
        if iterations == 1:
            _check(lib.ts_graph_capture_stream_iteration(target.handle, batch.handle, ctypes.byref(h)))
        else:
            _check(lib.ts_graph_capture_stream_iterations(target.handle, batch.handle, int(iterations),
                                                          ctypes.byref(h)))
        return cls(h, keep=batch)

    @classmethod
    def capture_batch_op(cls, target: Target, batch: Batch, op) -> "Graph":
        h = ctypes.c_void_p()
        _check(lib.ts_graph_capture_batch_op(target.handle, batch.handle, _op(op), ctypes.byref(h)))
        return cls(h, keep=batch)

    @classmethod
    def capture_arrays_iteration(cls, target: Target, a: Array, b: Array, c: Array, q: float = 3.0,
                                 iterations: int = 1) -> "Graph":
        """`iterations` consecutive plain iterations over a, b, c (4 nodes each)."""
        h = ctypes.c_void_p()
        if iterations == 1:
            _check(lib.ts_graph_capture_arrays_iteration(target.handle, a.handle, b.handle, c.handle, float(q),
                                                         ctypes.byref(h)))
        else:
            _check(lib.ts_graph_capture_arrays_iterations(target.handle, a.handle, b.handle, c.handle, float(q),
                                                          int(iterations), ctypes.byref(h)))
        return cls(h, keep=(a, b, c))

    def launch(self, target: Target, repeats: int = 1) -> None:
        _check(lib.ts_graph_launch(target.handle, self.handle, int(repeats)))

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.ts_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Event:
    """Completion marker on a target's stream (Listing 2's futures).

    timing=True makes an event for timing only (ts_event_create_timing): no
    system-scope release when recorded, so it disturbs the work it brackets
    less; synchronize the target before the host reads results."""

    def __init__(self, timing: bool = False):
        h = ctypes.c_void_p()
        _check((lib.ts_event_create_timing if timing else lib.ts_event_create)(ctypes.byref(h)))
        self.handle = h

    def record(self, target: Target) -> "Event":
        _check(lib.ts_event_record(self.handle, target.handle))
        return self

    def synchronize(self) -> None:
        _check(lib.ts_event_synchronize(self.handle))

    def query(self) -> bool:
        return _check(lib.ts_event_query(self.handle)) == 0

    def elapsed_ms(self, end: "Event") -> float:
        ms = ctypes.c_float()
        _check(lib.ts_event_elapsed_ms(self.handle, end.handle, ctypes.byref(ms)))
        return float(ms.value)

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.ts_event_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Transform:
    """dst[j] = expr(x[j], y[j], q): a C++ expression compiled at run time for
    the target's GPU (the executor runs any device callable, Section 4.2;
    e.g. the hello-world to_upper of Listing 3 over "u8" characters)."""

    def __init__(self, target: Target, expr: str, n_inputs: int = 1, dtype="f64"):
        h = ctypes.c_void_p()
        _check(lib.ts_transform_create(target.handle, expr.encode(), int(n_inputs), _dt(dtype), ctypes.byref(h)))
        self.handle = h
        self.n_inputs = int(n_inputs)
        self.dtype = dtype if isinstance(dtype, str) else DTYPE_NAMES[_dt(dtype)]

    def __call__(self, target: Target, x: Array, dst: Array, y: Array | None = None, q: float = 0.0) -> None:
        _check(lib.ts_transform_apply(target.handle, self.handle, x.handle, y.handle if y is not None else None,
                                      dst.handle, float(q)))

    def log(self) -> str:
        p = ctypes.c_char_p()
        _check(lib.ts_transform_log(self.handle, ctypes.byref(p)))
        return p.value.decode() if p.value else ""

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.ts_transform_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Future:
    """Completion of asynchronous work, made ready by a stream callback
    (the futures of Listing 2's async_execute)."""

    def __init__(self, handle):
        self.handle = handle

    def wait(self) -> None:
        _check(lib.ts_future_wait(self.handle))

    def ready(self) -> bool:
        return _check(lib.ts_future_ready(self.handle)) == 1

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib.ts_future_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_bytes(op, n: int, dtype: str = "f64") -> int:
    """Bytes the STREAM convention counts for one map over n elements."""
    name = op if isinstance(op, str) else list(OPS)[int(op)]
    return ARRAYS_MOVED[name] * int(n) * ELEM_SIZE[dtype]


load_default_tuning()
