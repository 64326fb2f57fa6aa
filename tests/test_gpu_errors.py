"""Error paths of the C ABI on a real device: every rule of the algorithm
calls returns its status (and a message) without launching anything, and
HIP failures come back as statuses."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

E_INVALID, E_SHAPE, E_DTYPE, E_PLACEMENT, E_ALIAS, E_DEVICE, E_OOM, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6, -7, -8


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    yield ts, torch, tgt
    tgt.synchronize()
    tgt.close()


def status(ts, fn):
    with pytest.raises(ts.TSError) as e:
        fn()
    assert e.value.message
    return e.value.status


def test_placement_and_wrapping(env):
    ts, torch, tgt = env
    host = np.zeros(16)
    h = ctypes.c_void_p()
    assert ts.lib.ts_array_wrap(tgt.handle, 0, host.ctypes.data, 16, ctypes.byref(h)) == E_PLACEMENT
    pinned = torch.zeros(16, dtype=torch.float64, pin_memory=True)
    assert ts.lib.ts_array_wrap(tgt.handle, 0, pinned.data_ptr(), 16, ctypes.byref(h)) == E_PLACEMENT
    dev = torch.zeros(16, dtype=torch.float64, device="cuda")
    assert ts.lib.ts_array_wrap(tgt.handle, 0, dev.data_ptr() + 4, 8, ctypes.byref(h)) == E_INVALID
    assert ts.lib.ts_array_wrap(tgt.handle, 0, None, 8, ctypes.byref(h)) == E_INVALID
    assert ts.lib.ts_array_wrap(tgt.handle, 7, dev.data_ptr(), 8, ctypes.byref(h)) == E_INVALID
    assert ts.lib.ts_array_wrap(tgt.handle, 0, None, 0, ctypes.byref(h)) == 0  # empty array
    ts.lib.ts_array_free(h)


def test_algorithm_rules(env):
    ts, torch, tgt = env
    t = torch.zeros(4096, dtype=torch.float64, device="cuda")
    a = ts.Array.wrap(tgt, t[0:1000])
    b = ts.Array.wrap(tgt, t[1024:2024])
    c = ts.Array.wrap(tgt, t[2048:3048])
    short = ts.Array.wrap(tgt, t[3072:3072 + 999])
    f32 = ts.Array.wrap(tgt, torch.zeros(1000, dtype=torch.float32, device="cuda"))
    overlap = ts.Array.wrap(tgt, t[1:1001])
    assert status(ts, lambda: ts.triad(tgt, a, b, short, 3.0)) == E_SHAPE
    assert status(ts, lambda: ts.add(tgt, a, short, c)) == E_SHAPE
    assert status(ts, lambda: ts.add(tgt, a, f32, c)) == E_DTYPE
    assert status(ts, lambda: ts.copy(tgt, a, f32)) == E_DTYPE
    assert status(ts, lambda: ts.triad(tgt, a, b, overlap, 3.0)) == E_ALIAS
    assert status(ts, lambda: ts.stream_iteration(tgt, a, overlap, c)) == E_ALIAS
    # an iteration whose third map would fail enqueues nothing: c keeps its values
    a.fill(5.0), c.fill(7.0)
    assert status(ts, lambda: ts.stream_iteration(tgt, a, short, c)) == E_SHAPE
    assert ts.checksum(tgt, c, 7.0)["mismatches"] == 0
    ts.copy(tgt, short, a)          # count = n of the first input: fewer elements is fine
    ts.triad(tgt, a, b, a, 3.0)     # exact in place
    ts.copy(tgt, ts.Array.wrap(tgt, t[0:0]), c)  # empty range: no launch
    out = np.zeros(2000)
    assert ts.lib.ts_copy_to_host(out.ctypes.data, a.handle, 1001) == E_SHAPE
    assert ts.lib.ts_copy_from_host(a.handle, out.ctypes.data, 1001) == E_SHAPE
    assert ts.lib.ts_fill_uniform(a.handle, 1, 1 << 16, 0) == E_INVALID
    assert ts.lib.ts_checksum(tgt.handle, a.handle, ctypes.c_double(0.0), None) == E_INVALID
    assert ts.lib.ts_mismatch_count(tgt.handle, a.handle, f32.handle, ctypes.byref(ctypes.c_uint64())) == E_DTYPE
    assert ts.lib.ts_mismatch_count(tgt.handle, a.handle, short.handle, ctypes.byref(ctypes.c_uint64())) == E_SHAPE
    tgt.synchronize()


def test_out_of_memory(env):
    ts, torch, tgt = env
    h = ctypes.c_void_p()
    rc = ts.lib.ts_array_alloc(tgt.handle, 0, 1 << 47, 0, ctypes.byref(h))  # 1 PiB
    assert rc == E_OOM, ts.last_error()
    # the device is still usable afterwards
    x = ts.Array.alloc(tgt, "f64", 1000).fill(2.0)
    assert ts.checksum(tgt, x, 2.0)["mismatches"] == 0


def test_graph_capture_needs_a_stream(env):
    ts, torch, tgt = env
    dflt = ts.Target(0, 0)  # the device's default stream
    a, b, c = (ts.Array.alloc(dflt, "f64", 100) for _ in range(3))
    assert status(ts, lambda: ts.Graph.capture_arrays_iteration(dflt, a, b, c)) == E_UNSUPPORTED
    for arr in (a, b, c):
        arr.fill(1.0)
    ts.stream_iteration(dflt, a, b, c)  # plain work on the default stream is fine
    dflt.synchronize()
    own = ts.Target(0, "own")
    assert own.stream_handle() != 0
    for bad in (0, -1, 4097):
        assert status(ts, lambda: ts.Graph.capture_arrays_iteration(own, a, b, c, iterations=bad)) == E_INVALID
    g = ts.Graph.capture_arrays_iteration(own, a, b, c)
    g.launch(own, 1)
    own.synchronize()
    # (1, 1, 1) -> (15, 3, 4) after the eager iteration, then a = 15 * 15 after the replay
    assert ts.checksum(own, a, 225.0)["mismatches"] == 0
    g.close()
    own.close()
    dflt.close()


def test_target_stream_choices_through_the_abi(env):
    """ts_target_create with NULL makes a non-blocking stream of the
    library's own (graph capture works on it); hipStreamLegacy binds the
    device's legacy default stream (the null handle; capture refused)."""
    ts, torch, tgt = env
    h = ctypes.c_void_p()
    assert ts.lib.ts_target_create(0, None, ctypes.byref(h)) == 0, ts.last_error()
    null_arg = ts.Target.__new__(ts.Target)
    null_arg.handle, null_arg.device, null_arg._torch_stream, null_arg._callbacks = h, 0, None, []
    assert null_arg.stream_handle() not in (0, ts.HIP_STREAM_LEGACY)
    a, b, c = (ts.Array.alloc(null_arg, "f64", 1000) for _ in range(3))
    for arr in (a, b, c):
        arr.fill(1.0)
    g = ts.Graph.capture_arrays_iteration(null_arg, a, b, c)
    g.launch(null_arg, 2)
    null_arg.synchronize()
    assert ts.checksum(null_arg, a, 225.0)["mismatches"] == 0  # (1, 1, 1) -> (15, 3, 4) -> a = 225
    g.close()
    h2 = ctypes.c_void_p()
    assert ts.lib.ts_target_create(0, ctypes.c_void_p(ts.HIP_STREAM_LEGACY), ctypes.byref(h2)) == 0
    legacy = ts.Target.__new__(ts.Target)
    legacy.handle, legacy.device, legacy._torch_stream, legacy._callbacks = h2, 0, None, []
    assert legacy.stream_handle() == 0
    assert status(ts, lambda: ts.Graph.capture_arrays_iteration(legacy, a, b, c)) == E_UNSUPPORTED
    legacy.close()
    null_arg.close()


def test_graph_refuses_freed_arrays(env):
    """A graph over library-owned arrays refuses to launch once one of them
    has been freed, instead of touching freed memory."""
    ts, torch, tgt = env
    own = ts.Target(0, "own")
    a, b, c = (ts.Array.alloc(own, "f64", 4099) for _ in range(3))
    for arr, v in zip((a, b, c), (1.0, 2.0, 0.0)):
        arr.fill(v)
    g = ts.Graph.capture_arrays_iteration(own, a, b, c, 3.0, iterations=2)
    g.launch(own, 1)
    own.synchronize()
    assert ts.checksum(own, a, 225.0)["mismatches"] == 0
    b.free()
    assert status(ts, lambda: g.launch(own, 1)) == E_INVALID
    assert "freed" in ts.last_error()
    g.close()
    a.free(), c.free()
    own.close()


def test_batch_errors(env):
    ts, torch, tgt = env
    host = np.zeros(64)
    with pytest.raises(ts.TSError) as e:
        ts.Batch(tgt, "f64", [(host.ctypes.data, host.ctypes.data, host.ctypes.data, 10, 1.0)])
    assert e.value.status == E_PLACEMENT
    dev = torch.zeros(128, dtype=torch.float64, device="cuda")  # every instance range lies inside it
    with pytest.raises(ts.TSError) as e:
        ts.Batch(tgt, "f64", [(dev.data_ptr(), 0, dev.data_ptr(), 10, 1.0)])
    assert e.value.status == E_INVALID
    b = ts.Batch(tgt, "f64", [(dev.data_ptr(), dev.data_ptr() + 256, dev.data_ptr() + 512 - 8, 4, 2.0)])
    with pytest.raises(ts.TSError):
        b.fill(tgt, 3, 1.0)
    with pytest.raises(ts.TSError):
        b.set_tile(12)
    with pytest.raises(ts.TSError):
        b.mismatch_count(tgt, 0, [1.0, 2.0])
    b.close()
    empty = ts.Batch(tgt, "f64", [])
    empty.op(tgt, "triad")
    assert empty.info()["tiles"] == 0
    empty.close()


def test_batch_and_wrap_refuse_overlap_and_overrun(env):
    """ts_batch_create refuses instances that share memory (TS_E_ALIAS) and
    arrays that run past the end of their device allocation (TS_E_SHAPE);
    ts_array_wrap refuses the overrun too.  Only the create and wrap calls
    run: nothing is launched on a refused batch."""
    ts, torch, tgt = env
    n = 1000
    A = ts.Array.alloc(tgt, "f64", 8 * n)  # one allocation of 8n doubles
    p = A.ptr()
    ok = [(p, p + 8 * n, p + 16 * n, n, 2.0), (p + 24 * n, p + 32 * n, p + 40 * n, n, 3.0)]
    b = ts.Batch(tgt, "f64", ok)
    b.close()
    b = ts.Batch(tgt, "f64", [(p, p, p + 16 * n, n, 2.0)])  # in place: the very same array
    b.close()
    cases = {
        "partial overlap inside an instance": ([(p, p + 8, p + 16 * n, n, 2.0)], E_ALIAS),
        "two instances share an array": ([ok[0], (p, p + 48 * n, p + 56 * n, n, 3.0)], E_ALIAS),
        "two instances overlap partly": ([ok[0], (p + 16 * n + 8, p + 48 * n, p + 56 * n, n, 3.0)], E_ALIAS),
        "array runs past its allocation": ([(p, p + 8 * n, p + 16 * n, n + (4 << 20), 2.0)], E_SHAPE),
    }
    for what, (descs, want) in cases.items():
        with pytest.raises(ts.TSError) as e:
            ts.Batch(tgt, "f64", descs)
        assert e.value.status == want, (what, e.value)
    h = ctypes.c_void_p()
    assert ts.lib.ts_array_wrap(tgt.handle, 0, p, 8 * n + (4 << 20), ctypes.byref(h)) == E_SHAPE
    assert "past the end" in ts.last_error()
    assert ts.lib.ts_array_wrap(tgt.handle, 0, p, 8 * n, ctypes.byref(h)) == 0
    ts.lib.ts_array_free(h)
    A.free()
