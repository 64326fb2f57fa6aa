"""The memory-system probe (ts_probe_bandwidth): what each mix of reads and
writes leaves in dst, for every launch shape the ceiling leg of the
benchmark searches, and the argument rules (refused without a launch)."""
import pytest

import bench
from gpu_util import say

pytestmark = pytest.mark.gpu

E_INVALID, E_SHAPE, E_PLACEMENT, E_ALIAS, E_UNSUPPORTED = -1, -2, -4, -5, -8
MARK = 0x5A5A5A5A


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    tgt = ts.Target(0, torch.cuda.Stream())
    yield ts, torch, tgt
    tgt.synchronize()
    tgt.close()


def _arrays(ts, torch, tgt, nbytes, seed):
    g = torch.Generator().manual_seed(seed)
    host = [torch.randint(0, 2 ** 62, (nbytes // 8,), dtype=torch.int64, generator=g) for _ in range(3)]
    dev = [h.cuda() for h in host]
    torch.cuda.synchronize()
    return host, dev, [ts.Array.wrap(tgt, d.view(torch.float64)) for d in dev]


@pytest.mark.parametrize("reads,writes", [(1, 0), (2, 0), (0, 1), (1, 1), (2, 1)])
def test_probe_results_every_shape(env, reads, writes):
    """dst = x, x ^ y or the mark pattern for every shape; with no write,
    dst keeps its contents (a lane stores only when the first word of its
    fold equals the mark, which these seeded inputs never give)."""
    ts, torch, tgt = env
    nbytes = 16 * 1024 * 4 * 6  # a multiple of every shape's vec_bytes * block * unroll
    host, dev, (X, Y, D) = _arrays(ts, torch, tgt, nbytes, reads * 10 + writes)
    for shape in bench.probe_shapes():
        cfg = dict(shape, reads=reads, writes=writes)
        dev[2].copy_(host[2].cuda())
        torch.cuda.synchronize()  # torch's stream is not ordered with the target's
        say(f"[probe {reads}r{writes}w {shape}]")
        ts.probe_bandwidth(tgt, cfg, X, Y, D, nbytes, MARK)
        tgt.synchronize()
        got = dev[2].cpu()
        if writes == 0:
            exp = host[2]
        elif reads == 0:
            exp = torch.full_like(host[2], (MARK << 32) | MARK)
        elif reads == 1:
            exp = host[0]
        else:
            exp = host[0] ^ host[1]
        assert torch.equal(got, exp), (reads, writes, shape)


@pytest.mark.parametrize("vb", [16, 8])
def test_probe_leaves_bytes_beyond_its_range(env, vb):
    """Only the first `bytes` bytes of dst are written."""
    ts, torch, tgt = env
    nbytes = vb * 256
    host, dev, (X, Y, D) = _arrays(ts, torch, tgt, 3 * 16 * 256, 3)
    say(f"[probe range vb={vb}]")
    ts.probe_bandwidth(tgt, {"reads": 2, "writes": 1, "block": 256, "unroll": 1, "nt_store": 1, "vec_bytes": vb},
                       X, Y, D, nbytes)
    tgt.synchronize()
    got = dev[2].cpu()
    k = nbytes // 8
    assert torch.equal(got[:k], host[0][:k] ^ host[1][:k]) and torch.equal(got[k:], host[2][k:])


def test_probe_rules(env):
    ts, torch, tgt = env
    t = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    X = ts.Array.wrap(tgt, t[0:8192])
    Y = ts.Array.wrap(tgt, t[8192:16384])
    D = ts.Array.wrap(tgt, t[16384:24576])
    odd = ts.Array.wrap(tgt, t[24577:24577 + 8192])  # 8-byte misaligned
    over = ts.Array.wrap(tgt, t[4096:4096 + 8192])  # overlaps X
    base = {"reads": 2, "writes": 1, "block": 256, "unroll": 1}

    def st(cfg, x, y, d, nbytes):
        with pytest.raises(ts.TSError) as e:
            ts.probe_bandwidth(tgt, cfg, x, y, d, nbytes)
        return e.value.status

    say("[probe rules]")
    assert st(dict(base, reads=0, writes=0), X, Y, D, 4096) == E_INVALID
    assert st(dict(base, reads=3), X, Y, D, 4096) == E_INVALID
    assert st(dict(base, block=96), X, Y, D, 4096 * 6) == E_INVALID
    assert st(dict(base, unroll=8), X, Y, D, 4096) == E_INVALID
    assert st(dict(base, vec_bytes=4), X, Y, D, 4096) == E_INVALID
    assert st(dict(base, vec_bytes=8), X, Y, D, 2048 + 8) == E_SHAPE  # not a multiple of 8 * block * unroll
    assert st(dict(base, lds_bytes=1 << 30), X, Y, D, 4096) == E_INVALID
    assert st(base, X, Y, D, 4096 + 16) == E_SHAPE  # not a multiple of 16 * block * unroll
    assert st(base, X, Y, D, 0) == E_SHAPE
    assert st(base, X, Y, D, 8192 * 8 * 2) == E_SHAPE  # longer than the arrays
    assert st(base, X, odd, D, 4096) == E_SHAPE
    assert st(base, X, Y, over, 8192 * 8) == E_ALIAS
    host = ts.Target.host([c for dom in ts.host_numa_domains() for c in dom][:1])
    try:
        with pytest.raises(ts.TSError) as e:
            ts.probe_bandwidth(host, base, X, Y, D, 4096)
        assert e.value.status == E_UNSUPPORTED
    finally:
        host.close()
    # refused calls launched nothing
    assert ts.checksum(tgt, D, 0.0)["mismatches"] == 0
