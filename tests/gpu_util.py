"""Helpers shared by the GPU tests: placing host arrays on the device through
the library, reading them back, and bitwise comparison (NaN matches NaN)."""
from __future__ import annotations

import sys

import numpy as np

import oracle

UINT = {"f64": np.uint64, "f32": np.uint32, "bf16": np.uint16, "f16": np.uint16}
ORACLE_DT = {"f64": oracle.F64, "f32": oracle.F32, "bf16": oracle.BF16, "f16": oracle.F16}


def say(*args):
    """Name the case before a GPU step (flushed, so a fault leaves a trace)."""
    print(*args, flush=True)
    sys.stdout.flush()


def device_array(ts, torch, tgt, host: np.ndarray, dtype: str, offset: int = 0, spare: int = 8):
    """Copy a host storage array into a fresh torch allocation at `offset`
    elements past its (>= 256-byte aligned) base and wrap it as an Array."""
    n = host.size
    t = torch.empty(n + offset + spare, dtype=ts.TORCH_DTYPES[dtype], device="cuda")
    assert t.data_ptr() % 256 == 0
    view = t[offset:offset + n]
    if n:
        src = host.view(np.int16) if host.dtype == np.uint16 else host
        view.copy_(torch.from_numpy(np.ascontiguousarray(src)).view(ts.TORCH_DTYPES[dtype]))
    torch.cuda.synchronize()
    return ts.Array.wrap(tgt, view)


def empty_array(ts, torch, tgt, n: int, dtype: str, offset: int = 0, fill_bits=None):
    t = torch.empty(n + offset + 8, dtype=ts.TORCH_DTYPES[dtype], device="cuda")
    view = t[offset:offset + n]
    if fill_bits is not None and n:
        view.view(torch.uint8).fill_(fill_bits)
    torch.cuda.synchronize()
    return ts.Array.wrap(tgt, view)


def widen(dtype: str, x: np.ndarray) -> np.ndarray:
    return oracle.widen_f64(ORACLE_DT[dtype], x)


def mismatches(got: np.ndarray, ref: np.ndarray, dtype: str) -> np.ndarray:
    """Indices where stored bits differ, NaN matching NaN."""
    g = got.view(UINT[dtype])
    r = ref.view(UINT[dtype])
    diff = g != r
    if diff.any():
        both_nan = np.isnan(widen(dtype, got)) & np.isnan(widen(dtype, ref))
        diff &= ~both_nan
    return np.nonzero(diff)[0]


def assert_same_bits(got, ref, dtype, what=""):
    bad = mismatches(got, ref, dtype)
    if bad.size:
        j = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} elements differ; first at {j}: "
                             f"got {widen(dtype, got[j:j+1])[0]!r} expected {widen(dtype, ref[j:j+1])[0]!r}")


# ---------------------------------------------------------------------------
# Whole-array comparison at full size
# ---------------------------------------------------------------------------
CHUNK = 1 << 24


def host_workers() -> int:
    """Threads for host-side oracle work: the CPUs this process may use,
    at most 16."""
    import os

    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _host_bits(buf, dtype: str) -> np.ndarray:
    import torch

    if dtype in ("bf16", "f16"):
        return buf.view(torch.int16).numpy().view(np.uint16)
    return buf.numpy()


def compare_whole(torch, views, dtype: str, expected, n: int, what: str = "", chunk: int = CHUNK):
    """Compare EVERY element of the device tensors `views` with the oracle.

    ``expected(start, stop)`` returns ``(arrays, info)``: one host storage
    array per view holding the oracle's results for elements [start, stop),
    and any per-chunk value the caller wants back.  It runs on a thread pool
    (the oracle's C calls and numpy's loops release the GIL), a few chunks
    ahead of the main thread, which copies each device chunk into a pinned
    host buffer and compares stored bits (NaN matches NaN).  The device work
    must be complete (synchronised) before the call.  Returns the infos in
    chunk order; raises AssertionError naming the first differing element."""
    import concurrent.futures as cf

    ranges = [(s, min(n, s + chunk)) for s in range(0, n, chunk)]
    if not ranges:
        return []
    workers = host_workers()
    pinned = torch.empty(min(chunk, n), dtype=views[0].dtype, pin_memory=True)
    infos = []
    with cf.ThreadPoolExecutor(workers) as pool:
        futs, nxt = {}, 0
        for i, (s, e) in enumerate(ranges):
            while nxt < len(ranges) and nxt <= i + workers + 1:
                futs[nxt] = pool.submit(expected, *ranges[nxt])
                nxt += 1
            arrays, info = futs.pop(i).result()
            infos.append(info)
            for k, (v, ref) in enumerate(zip(views, arrays)):
                buf = pinned[: e - s]
                buf.copy_(v[s:e])  # synchronous copy into pinned host memory
                got = _host_bits(buf, dtype)
                bad = mismatches(got, ref, dtype)
                if bad.size:
                    j = int(bad[0])
                    raise AssertionError(
                        f"{what}: array {k}: {bad.size} of {e - s} elements differ in chunk [{s}, {e}); "
                        f"first at {s + j}: got {widen(dtype, got[j:j + 1])[0]!r} "
                        f"expected {widen(dtype, ref[j:j + 1])[0]!r}")
    return infos
