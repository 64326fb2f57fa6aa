"""GPU parity of the batched ragged form: many (a, b, c, q) instances of
different lengths, one persistent launch per map, the four-map iteration
captured as a HIP graph.  Every instance must equal the oracle run on that
instance alone (the maps act element by element inside each instance, with
Listing 4's roles)."""
import numpy as np
import pytest

import oracle
import tsgen
from gpu_util import assert_same_bits, say

pytestmark = pytest.mark.gpu

OPS = ("copy", "scale", "add", "triad")


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2206_06302_amd as ts

    stream = torch.cuda.Stream()
    tgt = ts.Target(0, stream)
    yield ts, torch, tgt
    tgt.synchronize()
    tgt.close()
    torch.cuda.empty_cache()


class Pool:
    """One device allocation per array family; instance i's arrays start at
    offsets with chosen misalignments (in elements)."""

    def __init__(self, ts, torch, lens, dtype, mis=None):
        es = ts.ELEM_SIZE[dtype]
        self.dtype, self.lens = dtype, [int(n) for n in lens]
        mis = mis or [(0, 0, 0)] * len(lens)
        self.offs = [[], [], []]
        pos = [0, 0, 0]
        for n, m in zip(self.lens, mis):
            for k in range(3):
                start = (pos[k] + 31) // 32 * 32 + m[k]  # 256-byte slots, then the misalignment
                self.offs[k].append(start)
                pos[k] = start + n
        self.t = [torch.zeros(pos[k] + 64, dtype=ts.TORCH_DTYPES[dtype], device="cuda") for k in range(3)]
        self.es = es
        torch.cuda.synchronize()  # torch zero-fills on its own stream

    def ptr(self, k, i):
        return self.t[k].data_ptr() + self.offs[k][i] * self.es

    def descs(self, qs):
        return [(self.ptr(0, i), self.ptr(1, i), self.ptr(2, i), n, float(q))
                for i, (n, q) in enumerate(zip(self.lens, qs))]

    def view(self, k, i):
        return self.t[k][self.offs[k][i]:self.offs[k][i] + self.lens[i]]

    def upload(self, torch, k, i, host):
        if host.size:
            src = host.view(np.int16) if host.dtype == np.uint16 else host
            self.view(k, i).copy_(torch.from_numpy(np.ascontiguousarray(src)).view(self.t[k].dtype))

    def download(self, k, i):
        import torch

        v = self.view(k, i).cpu()
        if v.element_size() == 2:
            return v.view(torch.int16).numpy().view(np.uint16).copy()
        return v.numpy().copy()


def _lens(rng, count):
    base = [0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 31, 33, 1000, 4099, 16384, 16385, 65536 + 3]
    extra = list(rng.integers(1, 200000, count - len(base)))
    return base + extra


def _mis(rng, count, es):
    out = []
    for i in range(count):
        if i % 4 == 0:
            out.append((0, 0, 0))
        elif i % 4 == 1:
            m = int(rng.integers(0, 16 // es))
            out.append((m, m, m))
        else:
            out.append(tuple(int(v) for v in rng.integers(0, 16 // es, 3)))
    return out


def _host_instance(dtype, seed, i, n):
    return [tsgen.uniform_array(seed, tsgen.instance_stream(i, k), n, dtype) for k in range(3)]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_batched_ops_match_oracle(env, dtype):
    ts, torch, tgt = env
    rng = np.random.default_rng(42)
    count = 40
    lens = _lens(rng, count)
    pool = Pool(ts, torch, lens, dtype, _mis(rng, count, ts.ELEM_SIZE[dtype]))
    qs = tsgen.batched_scalars(5, count)
    host = []
    for i, n in enumerate(lens):
        h = _host_instance(dtype, 6, i, n)
        for k in range(3):
            pool.upload(torch, k, i, h[k])
        host.append(h)
    torch.cuda.synchronize()
    batch = ts.Batch(tgt, dtype, pool.descs(qs))
    info = batch.info()
    assert info["count"] == count and info["total_elems"] == sum(lens)
    for op in OPS:
        say(f"[batched {dtype} {op}] tiles={info['tiles']}")
        batch.op(tgt, op)
        tgt.synchronize()
        for i, n in enumerate(lens):
            a, b, c = host[i]
            xo = oracle.DTYPES[dtype]
            if op == "copy":
                oracle.op(xo, oracle.COPY, a, None, c, qs[i])
            elif op == "scale":
                oracle.op(xo, oracle.SCALE, c, None, b, qs[i])
            elif op == "add":
                oracle.op(xo, oracle.ADD, a, b, c, qs[i])
            else:
                oracle.op(xo, oracle.TRIAD, b, c, a, qs[i])
            for k in range(3):
                assert_same_bits(pool.download(k, i), host[i][k], dtype, f"{op} instance {i} (n={n}) array {k}")
    batch.close()


def test_batched_equals_plain_per_instance(env):
    ts, torch, tgt = env
    rng = np.random.default_rng(7)
    count = 24
    lens = _lens(rng, count)
    mis = _mis(rng, count, 8)
    p1 = Pool(ts, torch, lens, "f64", mis)
    p2 = Pool(ts, torch, lens, "f64", mis)
    qs = tsgen.batched_scalars(3, count)
    b1 = ts.Batch(tgt, "f64", p1.descs(qs))
    b2 = ts.Batch(tgt, "f64", p2.descs(qs))
    for k in range(3):
        b1.fill_uniform(tgt, k, 17)
        b2.fill_uniform(tgt, k, 17)
    say("[batched vs plain]")
    for _ in range(3):
        for op in OPS:
            b1.op(tgt, op)
            b2.op_plain(tgt, op)
    tgt.synchronize()
    for k in range(3):
        assert torch.equal(p1.t[k].view(torch.int64), p2.t[k].view(torch.int64))
    b1.close(), b2.close()


def test_batched_fill_matches_generator(env):
    ts, torch, tgt = env
    lens = [5, 1000, 17, 0, 33333]
    for dtype in ("f64", "bf16"):
        pool = Pool(ts, torch, lens, dtype, [(1, 0, 1), (0, 0, 0), (3, 3, 3), (0, 0, 0), (2, 1, 0)])
        batch = ts.Batch(tgt, dtype, pool.descs([1.0] * len(lens)))
        batch.fill_uniform(tgt, 1, 99)
        batch.fill(tgt, 2, 0.75)
        tgt.synchronize()
        for i, n in enumerate(lens):
            ref = tsgen.uniform_array(99, tsgen.instance_stream(i, 1), n, dtype)
            assert_same_bits(pool.download(1, i), ref, dtype, f"fill_uniform instance {i}")
            assert_same_bits(pool.download(2, i), tsgen.narrow(np.full(n, 0.75), dtype), dtype, "fill")
        batch.close()


def test_graph_iteration_matches_eager_and_closed_form(env):
    """The captured four-map iteration, replayed with eager work and
    synchronisations between replays, equals eager iterations; from
    (1, 2, 0) every element of instance i equals the scalar chain with q_i."""
    ts, torch, tgt = env
    rng = np.random.default_rng(3)
    count = 32
    lens = _lens(rng, count)
    mis = _mis(rng, count, 8)
    pg = Pool(ts, torch, lens, "f64", mis)
    pe = Pool(ts, torch, lens, "f64", mis)
    qs = tsgen.batched_scalars(5, count)
    bg = ts.Batch(tgt, "f64", pg.descs(qs))
    be = ts.Batch(tgt, "f64", pe.descs(qs))
    for b in (bg, be):
        b.fill(tgt, 0, 1.0), b.fill(tgt, 1, 2.0), b.fill(tgt, 2, 0.0)
    say("[graph iteration]")
    g = ts.Graph.capture_stream_iteration(tgt, bg)
    done = 0
    for rep in (1, 3, 6):
        g.launch(tgt, rep)
        for _ in range(rep):
            for op in OPS:
                be.op(tgt, op)
        done += rep
        tgt.synchronize()
        for k in range(3):
            assert torch.equal(pg.t[k].view(torch.int64), pe.t[k].view(torch.int64)), (rep, k)
        exp = [oracle.stream_scalar_f64(1.0, 2.0, 0.0, float(q), done) for q in qs]
        for k in range(3):
            counts = bg.mismatch_count(tgt, k, np.array([e[k] for e in exp]))
            assert counts.sum() == 0, (done, k, np.nonzero(counts)[0][:5])
    g.close()
    g1 = ts.Graph.capture_batch_op(tgt, bg, "triad")
    g1.launch(tgt, 2)
    be.op(tgt, "triad"), be.op(tgt, "triad")
    tgt.synchronize()
    assert torch.equal(pg.t[0].view(torch.int64), pe.t[0].view(torch.int64))
    g1.close(), bg.close(), be.close()


def test_multi_iteration_batched_graph(env):
    """Five batched iterations captured as one 20-node graph, replayed twice:
    every instance follows the scalar chain with its own q for 10 iterations."""
    ts, torch, tgt = env
    rng = np.random.default_rng(17)
    count = 24
    lens = _lens(rng, count)
    pool = Pool(ts, torch, lens, "f64", _mis(rng, count, 8))
    qs = tsgen.batched_scalars(6, count)
    batch = ts.Batch(tgt, "f64", pool.descs(qs))
    batch.fill(tgt, 0, 1.0), batch.fill(tgt, 1, 2.0), batch.fill(tgt, 2, 0.0)
    say("[multi-iteration batched graph]")
    g = ts.Graph.capture_stream_iteration(tgt, batch, iterations=5)
    g.launch(tgt, 1)
    tgt.synchronize()
    g.launch(tgt, 1)
    tgt.synchronize()
    g.close()
    exp = [oracle.stream_scalar_f64(1.0, 2.0, 0.0, float(q), 10) for q in qs]
    for k in range(3):
        counts = batch.mismatch_count(tgt, k, np.array([e[k] for e in exp]))
        assert counts.sum() == 0, (k, np.nonzero(counts)[0][:5])
    batch.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_batched_fill_and_count_over_tiles(env, dtype):
    """Fills and mismatch counts read and write each tile as an element-wise
    head, 16-byte vectors and a tail: with tiles that start off the vector
    grid, every misalignment of each array and instances shorter than one
    vector, the fills give the generator's bits, nothing outside the
    instances is written, and the counts equal numpy's."""
    ts, torch, tgt = env
    rng = np.random.default_rng(21)
    es = ts.ELEM_SIZE[dtype]
    lens = [1, 2, 3, 5, 7, 8, 9, 15, 17, 100, 513, 1000, 4099, 20001]
    mis = [tuple(int(v) for v in rng.integers(0, 16 // es, 3)) for _ in lens]
    for tile in (8, 24, 512, 4096):
        say(f"[batched fill/count {dtype} tile {tile}]")
        pool = Pool(ts, torch, lens, dtype, mis)
        batch = ts.Batch(tgt, dtype, pool.descs([1.0] * len(lens)))
        batch.set_tile(tile)
        batch.fill_uniform(tgt, 0, 31)
        batch.fill(tgt, 1, -0.375)
        batch.fill_uniform(tgt, 2, 32)
        tgt.synchronize()
        inside = [np.zeros(pool.t[k].numel(), bool) for k in range(3)]
        for i, n in enumerate(lens):
            for k in range(3):
                inside[k][pool.offs[k][i]:pool.offs[k][i] + n] = True
            assert_same_bits(pool.download(0, i), tsgen.uniform_array(31, tsgen.instance_stream(i, 0), n, dtype),
                             dtype, f"uniform a[{i}]")
            assert_same_bits(pool.download(1, i), tsgen.narrow(np.full(n, -0.375), dtype), dtype, f"b[{i}]")
            assert_same_bits(pool.download(2, i), tsgen.uniform_array(32, tsgen.instance_stream(i, 2), n, dtype),
                             dtype, f"uniform c[{i}]")
        for k in range(3):
            whole = pool.t[k].view(torch.int16 if es == 2 else torch.int32 if es == 4 else torch.int64).cpu().numpy()
            assert not whole[~inside[k]].any(), f"array {k}: a write outside the instances"
        # plant mismatches at the first, a middle and the last element of some instances
        want = np.zeros(len(lens), np.uint64)
        for i, n in enumerate(lens):
            if i % 2:
                continue
            for j in sorted({0, n // 2, n - 1}):
                pool.view(1, i)[j] = 0.5
                want[i] += 1
        torch.cuda.synchronize()
        exp = np.full(len(lens), -0.375)  # exact in every storage type
        assert list(batch.mismatch_count(tgt, 1, exp)) == list(want)
        assert list(batch.mismatch_count(tgt, 1, exp + 1.0)) == lens
        batch.close()


def test_batch_mismatch_count_counts(env):
    ts, torch, tgt = env
    lens = [10, 0, 5000, 3]
    pool = Pool(ts, torch, lens, "f64")
    batch = ts.Batch(tgt, "f64", pool.descs([1.0] * 4))
    batch.fill(tgt, 0, 2.5)
    tgt.synchronize()
    pool.view(0, 2)[17] = 1.0
    pool.view(0, 2)[4999] = float("nan")
    torch.cuda.synchronize()
    counts = batch.mismatch_count(tgt, 0, np.array([2.5, 0.0, 2.5, 7.0]))
    assert list(counts) == [0, 0, 2, 3]
    batch.close()


def test_batch_tile_sizes_do_not_change_results(env):
    ts, torch, tgt = env
    rng = np.random.default_rng(11)
    lens = _lens(rng, 20)
    mis = _mis(rng, 20, 8)
    ref_pool = Pool(ts, torch, lens, "f64", mis)
    qs = tsgen.batched_scalars(8, 20)
    ref = ts.Batch(tgt, "f64", ref_pool.descs(qs))
    for k in range(3):
        ref.fill_uniform(tgt, k, 4)
    for op in OPS:
        ref.op_plain(tgt, op)
    for tile in (8, 24, 4096, 16384, 1 << 20):
        pool = Pool(ts, torch, lens, "f64", mis)
        b = ts.Batch(tgt, "f64", pool.descs(qs))
        b.set_tile(tile)
        for k in range(3):
            b.fill_uniform(tgt, k, 4)
        say(f"[tile {tile}]")
        for op in OPS:
            b.op(tgt, op)
        tgt.synchronize()
        for k in range(3):
            assert torch.equal(pool.t[k].view(torch.int64), ref_pool.t[k].view(torch.int64)), (tile, k)
        b.close()
    ref.close()


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_batch_launch_shapes_do_not_change_results(env, dtype):
    """One workgroup per tile (grid_per_cu 0) and persistent grids of several
    sizes give the per-instance plain launches' results bit for bit."""
    ts, torch, tgt = env
    rng = np.random.default_rng(12)
    lens = _lens(rng, 24)
    mis = _mis(rng, 24, ts.ELEM_SIZE[dtype])
    qs = tsgen.batched_scalars(9, 24)
    ref_pool = Pool(ts, torch, lens, dtype, mis)
    ref = ts.Batch(tgt, dtype, ref_pool.descs(qs))
    for k in range(3):
        ref.fill_uniform(tgt, k, 6)
    for op in OPS:
        ref.op_plain(tgt, op)
    # (grid_per_cu, block, unroll, tile, tiles per workgroup, workgroups per tile, vector bytes)
    shapes = [(0, 256, 1, 24, 1, 1, 16), (0, 1024, 4, 4096, 1, 1, 16), (0, 512, 2, 2048, 1, 1, 16),
              (1, 1024, 8, 16384, 1, 1, 16), (64, 64, 1, 8, 1, 1, 16), (0, 256, 1, 24, 8, 1, 16),
              (0, 512, 2, 1024, 4, 1, 16), (2, 256, 2, 512, 2, 1, 16), (0, 64, 1, 8, 4, 1, 16),
              # one-wave workgroups sharing tiles: tiles smaller and larger than their pieces
              (0, 64, 1, 2048, 1, 32, 8), (0, 64, 1, 1024, 1, 16, 16), (0, 64, 1, 24, 1, 8, 8),
              (0, 64, 1, 8192, 1, 2, 16)]
    try:
        for grid, block, unroll, tile, per_wg, pieces, vb in shapes:
            cfg = {"block": block, "unroll": unroll, "vec_bytes": vb, "nt_load": 1, "nt_store": 1,
                   "grid_per_cu": grid, "tile_elems": tile, "tiles_per_wg": per_wg, "wgs_per_tile": pieces}
            for op in OPS:
                ts.set_kernel_cfg(op, dtype, cfg, batched=True)
            pool = Pool(ts, torch, lens, dtype, mis)
            b = ts.Batch(tgt, dtype, pool.descs(qs))
            b.set_tile(tile)
            for k in range(3):
                b.fill_uniform(tgt, k, 6)
            say(f"[launch shape grid_per_cu={grid} block={block} U{unroll} VB{vb} tile={tile} x{per_wg} "
                f"/{pieces} {dtype}]")
            for op in OPS:
                b.op(tgt, op)
            tgt.synchronize()
            for k in range(3):
                assert torch.equal(pool.t[k].view(torch.int16), ref_pool.t[k].view(torch.int16)), (grid, tile, k)
            b.close()
    finally:
        for op in OPS:
            ts.set_kernel_cfg(op, dtype, None, batched=True)
    ref.close()


def test_each_map_runs_on_its_own_tiles(env):
    """Configurations with a different tile size per map give one batch
    several tile plans; eager maps and a captured iteration both equal the
    per-instance plain launches bit for bit."""
    ts, torch, tgt = env
    rng = np.random.default_rng(13)
    lens = _lens(rng, 24)
    mis = _mis(rng, 24, 8)
    qs = tsgen.batched_scalars(10, 24)
    cfgs = {"copy": (0, 512, 1, 1024), "scale": (8, 1024, 4, 16384), "add": (0, 1024, 2, 4096),
            "triad": (0, 256, 1, 24)}
    ref_pool = Pool(ts, torch, lens, "f64", mis)
    ref = ts.Batch(tgt, "f64", ref_pool.descs(qs))
    for k in range(3):
        ref.fill_uniform(tgt, k, 7)
    try:
        for op, (grid, block, unroll, tile) in cfgs.items():
            ts.set_kernel_cfg(op, "f64", {"block": block, "unroll": unroll, "vec_bytes": 16, "nt_load": 1,
                                          "nt_store": 1, "grid_per_cu": grid, "tile_elems": tile}, batched=True)
        pool = Pool(ts, torch, lens, "f64", mis)
        b = ts.Batch(tgt, "f64", pool.descs(qs))
        assert b.info()["tile_elems"] == 24  # the primary plan follows the triad
        for k in range(3):
            b.fill_uniform(tgt, k, 7)
        say("[per-map tile plans]")
        for op in OPS:
            b.op(tgt, op)
            ref.op_plain(tgt, op)
        g = ts.Graph.capture_stream_iteration(tgt, b, iterations=2)
        g.launch(tgt, 1)
        for _ in range(2):
            for op in OPS:
                ref.op_plain(tgt, op)
        tgt.synchronize()
        for k in range(3):
            assert torch.equal(pool.t[k].view(torch.int64), ref_pool.t[k].view(torch.int64)), k
        g.close()
        b.close()
    finally:
        for op in OPS:
            ts.set_kernel_cfg(op, "f64", None, batched=True)
    ref.close()


def test_graph_refuses_a_replanned_or_destroyed_batch(env):
    """A re-plan frees the tile tables a captured graph points to: launching
    that graph afterwards is refused on the host."""
    ts, torch, tgt = env
    lens = [1000, 5000, 17]
    pool = Pool(ts, torch, lens, "f64")
    b = ts.Batch(tgt, "f64", pool.descs([2.0] * 3))
    for k, v in enumerate((1.0, 2.0, 0.0)):
        b.fill(tgt, k, v)
    g = ts.Graph.capture_stream_iteration(tgt, b)
    g.launch(tgt, 1)
    tgt.synchronize()
    b.set_tile(4096)
    with pytest.raises(ts.TSError) as e:
        g.launch(tgt, 1)
    assert e.value.status == -1 and "re-planned" in e.value.message
    g.close()
    g2 = ts.Graph.capture_batch_op(tgt, b, "triad")
    g2.launch(tgt, 1)
    tgt.synchronize()
    b.close()
    with pytest.raises(ts.TSError) as e:
        g2.launch(tgt, 1)
    assert e.value.status == -1
    g2.close()
