"""The allocation-free checksum (ts_checksum_noalloc) against ts_checksum.

Both run the same two reduction kernels over the same tree; the
allocation-free form keeps its partial sums in a fixed per-GPU device array
and stores the result in caller-owned device memory.  Its four results must
equal ts_checksum's bit for bit, on consecutive calls with a smaller input
second (so parts left in the fixed array by the first call must not leak
into the second), and on an empty array."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _result(out):
    """The 32-byte ts_checksum_out at the start of the uint8 tensor `out`."""
    raw = out[:32].cpu().numpy()
    f = raw[:24].view(np.float64)
    return float(f[0]), float(f[1]), float(f[2]), int(raw[24:32].view(np.uint64)[0])


def _bits(v):
    return np.float64(v).view(np.uint64)


def test_noalloc_checksum_equals_checksum_on_consecutive_calls():
    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    out = torch.full((64,), 0xAB, dtype=torch.uint8, device="cuda")  # a poisoned result slot
    torch.cuda.synchronize()
    # (storage type, n, element offset from an aligned base, expected value);
    # the second is far smaller than the first, the third empty.
    cases = [("f64", (1 << 22) + 13, 1, 0.25), ("f32", 1003, 1, 0.5), ("f64", 0, 0, 1.0)]
    for dtype, n, off, expected in cases:
        say(f"[noalloc checksum {dtype} n={n} offset={off}]")
        base = torch.empty(n + off + 8, dtype=ts.TORCH_DTYPES[dtype], device="cuda")
        view = base[off:off + n]
        torch.cuda.synchronize()
        X = ts.Array.wrap(tgt, view)
        if n:
            X.fill_uniform(31, 0)
            ts.Array.wrap(tgt, view[: n // 3]).fill(expected)  # a third of the elements match exactly
        ref = ts.checksum(tgt, X, expected)
        ts.checksum_noalloc(tgt, X, expected, out.data_ptr())
        tgt.synchronize()
        got = _result(out)
        want = (ref["sum"], ref["abs_dev_sum"], ref["max_abs_dev"], ref["mismatches"])
        for g, w, name in zip(got[:3], want[:3], ("sum", "abs_dev_sum", "max_abs_dev")):
            assert _bits(g) == _bits(w), (dtype, n, name, g, w)
        assert got[3] == want[3], (dtype, n, got[3], want[3])
        # The exact parts of the result against the host copy of the array.
        host = view.cpu().numpy().astype(np.float64)
        assert got[3] == int(np.count_nonzero(host != expected))
        assert got[2] == (float(np.max(np.abs(host - expected))) if n else 0.0)
        if n:
            assert got[3] == n - n // 3
        del X, view, base
    tgt.close()


def test_noalloc_checksum_refuses_bad_output():
    """dev_out must be device memory of the target's GPU, aligned, and must
    not overlap the array; nothing is launched when it is refused."""
    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    t = torch.zeros(4096, dtype=torch.float64, device="cuda")
    out = torch.zeros(64, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    X = ts.Array.wrap(tgt, t)
    host = np.zeros(8, np.float64)
    with pytest.raises(ts.TSError) as e:
        ts.checksum_noalloc(tgt, X, 0.0, host.ctypes.data)
    assert e.value.status == -4
    with pytest.raises(ts.TSError) as e:
        ts.checksum_noalloc(tgt, X, 0.0, out.data_ptr() + 4)
    assert e.value.status == -1
    with pytest.raises(ts.TSError) as e:
        ts.checksum_noalloc(tgt, X, 0.0, t.data_ptr() + 64)
    assert e.value.status == -5
    tgt.synchronize()
    tgt.close()
