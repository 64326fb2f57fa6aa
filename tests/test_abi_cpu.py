"""CPU-side tests of the C-ABI library: exports, argument checks that need no
device, the tuning table, and the GPU-free launch/batch planning rules."""
import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tstream.h")
LIBPATH = os.path.join(ROOT, "paper_2206_06302_amd", "libtstream.so")
CSRC = os.path.join(ROOT, "paper_2206_06302_amd", "csrc")

TS_OK, TS_E_INVALID, TS_E_SHAPE, TS_E_DTYPE, TS_E_PLACEMENT, TS_E_ALIAS, TS_E_DEVICE = 0, -1, -2, -3, -4, -5, -6


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"TS_API\s+[^;(]*?\b(ts_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def raw():
    if not os.path.exists(LIBPATH):
        pytest.fail("libtstream.so is not built (run __graft_entry__.build())")
    import torch  # noqa: F401  (load torch's HIP runtime first, as the binding does)
    return ctypes.CDLL(LIBPATH)


@pytest.fixture(scope="module")
def ts():
    import paper_2206_06302_amd as ts
    return ts


def test_every_declared_symbol_is_exported(raw):
    names = declared_functions()
    assert len(names) >= 50
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing


def test_no_undeclared_exports():
    """The dynamic symbol table holds the header's functions and nothing else
    (kernel stubs, helpers and template instances stay local)."""
    out = subprocess.run(["nm", "-D", "--defined-only", LIBPATH], capture_output=True, text=True, check=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if l.strip())
    assert exported == declared_functions()


def test_binding_covers_every_function(ts):
    from paper_2206_06302_amd import _lib
    assert sorted(_lib.PROTOTYPES) == declared_functions()


def test_version_and_errors(ts):
    assert ts.version() == (2, 1)
    L = ts.lib
    assert L.ts_copy(None, None, None) == TS_E_INVALID
    assert "invalid" in ts.last_error()
    assert L.ts_triad(None, None, None, None, ctypes.c_double(3.0)) == TS_E_INVALID
    assert L.ts_target_synchronize(None) == TS_E_INVALID
    assert L.ts_array_info(None, None, None, None) == TS_E_INVALID
    assert L.ts_version(None, None) == TS_E_INVALID
    # destroy/free accept NULL as a no-op and never fail on it
    for fn in ("ts_target_destroy", "ts_array_free", "ts_batch_destroy", "ts_graph_destroy", "ts_event_destroy",
               "ts_future_destroy"):
        assert getattr(L, fn)(None) == TS_OK
    assert L.ts_batch_op(None, None, 3) == TS_E_INVALID
    assert L.ts_graph_launch(None, None, 1) == TS_E_INVALID
    assert L.ts_event_query(None) == TS_E_INVALID
    assert L.ts_event_create(None) == TS_E_INVALID
    assert L.ts_event_create_timing(None) == TS_E_INVALID
    assert L.ts_future_wait(None) == TS_E_INVALID
    assert L.ts_future_ready(None) == TS_E_INVALID
    assert L.ts_future_destroy(None) == TS_OK
    assert L.ts_target_async(None, None) == TS_E_INVALID
    assert L.ts_transform_create(None, b"x", 1, 0, None) == TS_E_INVALID
    assert L.ts_transform_apply(None, None, None, None, None, ctypes.c_double(0.0)) == TS_E_INVALID
    assert L.ts_transform_destroy(None) == TS_OK


def test_target_create_without_gpu_reports_device_error(ts):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = ts.lib.ts_target_create(0, None, ctypes.byref(h))
    assert rc == TS_E_DEVICE and "GPU" in ts.last_error()
    assert ts.lib.ts_target_create(0, None, None) == TS_E_INVALID


# --------------------------------------------------------------- tuning table
def test_tune_table_roundtrip(ts, tmp_path):
    ts.tune_cache_clear()
    base = ts.get_kernel_cfg("triad", "f64", 1 << 27)
    assert base["vec_bytes"] == 16 and base["grid_per_cu"] == 0
    p = tmp_path / "t.json"
    doc = {"format": "tstream-tune", "version": 1, "entries": [
        {"op": "triad", "dtype": "f64", "bucket": 27, "align": 0, "batched": 0, "block": 512, "unroll": 2,
         "vec_bytes": 16, "nt_load": 1, "nt_store": 1, "grid_per_cu": 4, "tile_elems": 0, "bytes_per_s": 6.9e12},
        {"op": "copy", "dtype": "bf16", "bucket": 20, "align": 1, "batched": 0, "block": 1024, "unroll": 8,
         "vec_bytes": 8, "nt_load": 0, "nt_store": 0, "grid_per_cu": 0, "tile_elems": 0},
        {"op": "triad", "dtype": "f64", "bucket": 32, "align": 0, "batched": 1, "block": 256, "unroll": 4,
         "vec_bytes": 16, "nt_load": 0, "nt_store": 1, "grid_per_cu": 8, "tile_elems": 65536}]}
    p.write_text(json.dumps(doc))
    ts.tune_cache_load(str(p))
    c = ts.get_kernel_cfg("triad", "f64", 1 << 27)
    assert (c["block"], c["unroll"], c["nt_load"], c["grid_per_cu"]) == (512, 2, 1, 4)
    # nearest size bucket with the same op/dtype/alignment/batched fields
    assert ts.get_kernel_cfg("triad", "f64", 1 << 16)["block"] == 512
    assert ts.get_kernel_cfg("triad", "f64", 1 << 27, align_class=1)["block"] == 256  # default
    assert ts.get_kernel_cfg("copy", "bf16", 1 << 20, align_class=1)["vec_bytes"] == 8
    assert ts.get_kernel_cfg("triad", "f64", 4 << 30, batched=True)["tile_elems"] == 65536
    # mixed misalignment falls back to the element-wise width by default
    assert ts.get_kernel_cfg("add", "f32", 1000, align_class=2)["vec_bytes"] == 4
    # an entry without tiles_per_wg (written before the field) holds one tile per workgroup
    assert ts.get_kernel_cfg("triad", "f64", 4 << 30, batched=True)["tiles_per_wg"] == 1
    doc["entries"].append({"op": "copy", "dtype": "f64", "bucket": 32, "align": 0, "batched": 1, "block": 256,
                           "unroll": 1, "vec_bytes": 16, "nt_load": 1, "nt_store": 1, "grid_per_cu": 0,
                           "tile_elems": 512, "tiles_per_wg": 4})
    p.write_text(json.dumps(doc))
    ts.tune_cache_load(str(p))
    assert ts.get_kernel_cfg("copy", "f64", 4 << 30, batched=True)["tiles_per_wg"] == 4
    q = tmp_path / "u.json"
    ts.tune_cache_save(str(q))
    saved = json.loads(q.read_text())
    assert saved["format"] == "tstream-tune" and len(saved["entries"]) == 4
    assert {e["op"]: e["tiles_per_wg"] for e in saved["entries"] if e["batched"]} == {"triad": 1, "copy": 4}
    assert all(e["record_ahead"] == 0 for e in saved["entries"])
    ts.tune_cache_clear()
    ts.tune_cache_load(str(q))
    assert ts.get_kernel_cfg("triad", "f64", 1 << 27)["block"] == 512
    assert ts.get_kernel_cfg("copy", "f64", 4 << 30, batched=True)["tiles_per_wg"] == 4
    ts.tune_cache_clear()


@pytest.mark.parametrize("text", [
    "", "{", "[]", '{"format": "other", "version": 1, "entries": []}',
    '{"format": "tstream-tune", "version": 2, "entries": []}',
    '{"format": "tstream-tune", "version": 1}',
    '{"format": "tstream-tune", "version": 1, "entries": [{"op": "triad"}]}',
    '{"format": "tstream-tune", "version": 1, "entries": [{"op": "fma", "dtype": "f64", "bucket": 1, "align": 0, '
    '"batched": 0, "block": 256, "unroll": 4, "vec_bytes": 16, "nt_load": 0, "nt_store": 0, "grid_per_cu": 0, '
    '"tile_elems": 0}]}',
    '{"format": "tstream-tune", "version": 1, "entries": [{"op": "copy", "dtype": "f64", "bucket": 1, "align": 0, '
    '"batched": 0, "block": 100, "unroll": 4, "vec_bytes": 16, "nt_load": 0, "nt_store": 0, "grid_per_cu": 0, '
    '"tile_elems": 0}]}',
    '{"format": "tstream-tune", "version": 1, "entries": []} trailing',
])
def test_tune_table_rejects_bad_files(ts, tmp_path, text):
    ts.tune_cache_clear()
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"format": "tstream-tune", "version": 1, "entries": [
        {"op": "add", "dtype": "f32", "bucket": 10, "align": 0, "batched": 0, "block": 128, "unroll": 1,
         "vec_bytes": 16, "nt_load": 0, "nt_store": 0, "grid_per_cu": 2, "tile_elems": 0}]}))
    ts.tune_cache_load(str(good))
    bad = tmp_path / "bad.json"
    bad.write_text(text)
    with pytest.raises(ts.TSError) as e:
        ts.tune_cache_load(str(bad))
    assert e.value.status == TS_E_INVALID
    assert ts.get_kernel_cfg("add", "f32", 1024)["block"] == 128  # table unchanged
    with pytest.raises(ts.TSError):
        ts.tune_cache_load(str(tmp_path / "missing.json"))
    ts.tune_cache_clear()


def test_forced_configuration(ts):
    before = ts.get_kernel_cfg("scale", "f16", 5)
    ts.set_kernel_cfg("scale", "f16", {"block": 1024, "unroll": 8, "vec_bytes": 8, "nt_load": 1,
                                       "nt_store": 0, "grid_per_cu": 2})
    assert ts.get_kernel_cfg("scale", "f16", 5)["block"] == 1024
    ts.set_kernel_cfg("scale", "f16", None)
    assert ts.get_kernel_cfg("scale", "f16", 5) == before
    for bad in ({"block": 96}, {"unroll": 3}, {"vec_bytes": 32}, {"nt_load": 2}, {"grid_per_cu": -1}):
        cfg = {"block": 256, "unroll": 4, "vec_bytes": 16, "nt_load": 0, "nt_store": 0, "grid_per_cu": 0}
        cfg.update(bad)
        with pytest.raises(ts.TSError):
            ts.set_kernel_cfg("copy", "f64", cfg)
    with pytest.raises(ts.TSError):  # batched kernels require 16-byte vectors
        ts.set_kernel_cfg("copy", "f64", {"block": 256, "unroll": 1, "vec_bytes": 8, "grid_per_cu": 4,
                                          "tile_elems": 8192}, batched=True)
    for bad in ({"grid_per_cu": -1}, {"grid_per_cu": 65}, {"tile_elems": 12}):
        cfg = {"block": 1024, "unroll": 4, "vec_bytes": 16, "nt_load": 1, "nt_store": 1, "grid_per_cu": 0,
               "tile_elems": 4096}
        cfg.update(bad)
        with pytest.raises(ts.TSError):
            ts.set_kernel_cfg("copy", "f64", cfg, batched=True)
    # several tiles per workgroup: 1, 2, 4 or 8, with unroll 1 or 2; plain kernels take 0 or 1
    for bad in ({"tiles_per_wg": 3}, {"tiles_per_wg": 16}, {"tiles_per_wg": -1},
                {"tiles_per_wg": 2, "unroll": 4}, {"record_ahead": 2}, {"record_ahead": 1, "tiles_per_wg": 2},
                {"record_ahead": 1, "grid_per_cu": 4}, {"wgs_per_tile": 3}, {"wgs_per_tile": 256},
                {"wgs_per_tile": 16}, {"wgs_per_tile": 16, "block": 64, "unroll": 2},
                {"wgs_per_tile": 16, "block": 64, "record_ahead": 1},
                {"wgs_per_tile": 16, "block": 64, "vec_bytes": 4}, {"vec_bytes": 8}):
        cfg = {"block": 256, "unroll": 1, "vec_bytes": 16, "nt_load": 1, "nt_store": 1, "grid_per_cu": 0,
               "tile_elems": 512}
        cfg.update(bad)
        with pytest.raises(ts.TSError):
            ts.set_kernel_cfg("copy", "f64", cfg, batched=True)
    with pytest.raises(ts.TSError):
        ts.set_kernel_cfg("copy", "f64", {"block": 256, "unroll": 1, "vec_bytes": 16, "tiles_per_wg": 2})
    with pytest.raises(ts.TSError):
        ts.set_kernel_cfg("copy", "f64", {"block": 256, "unroll": 1, "vec_bytes": 16, "record_ahead": 1})
    ts.set_kernel_cfg("scale", "f64", {"block": 256, "unroll": 1, "vec_bytes": 16, "nt_load": 1, "nt_store": 1,
                                       "grid_per_cu": 0, "tile_elems": 512, "record_ahead": 1}, batched=True)
    assert ts.get_kernel_cfg("scale", "f64", 1 << 30, batched=True)["record_ahead"] == 1
    ts.set_kernel_cfg("scale", "f64", None, batched=True)
    ts.set_kernel_cfg("add", "f64", {"block": 256, "unroll": 2, "vec_bytes": 16, "nt_load": 1, "nt_store": 1,
                                     "grid_per_cu": 0, "tile_elems": 1024, "tiles_per_wg": 8}, batched=True)
    assert ts.get_kernel_cfg("add", "f64", 1 << 30, batched=True)["tiles_per_wg"] == 8
    ts.set_kernel_cfg("add", "f64", None, batched=True)
    ts.set_kernel_cfg("triad", "f64", {"block": 64, "unroll": 1, "vec_bytes": 8, "nt_load": 1, "nt_store": 1,
                                       "grid_per_cu": 0, "tile_elems": 2048, "wgs_per_tile": 32}, batched=True)
    assert ts.get_kernel_cfg("triad", "f64", 1 << 30, batched=True)["wgs_per_tile"] == 32
    ts.set_kernel_cfg("triad", "f64", None, batched=True)
    with pytest.raises(ts.TSError):  # plain kernels take wgs_per_tile 0 or 1
        ts.set_kernel_cfg("copy", "f64", {"block": 64, "unroll": 1, "vec_bytes": 8, "wgs_per_tile": 2})
    # grid_per_cu 0 on the batched path: one workgroup per tile
    ts.set_kernel_cfg("copy", "f64", {"block": 1024, "unroll": 4, "vec_bytes": 16, "nt_load": 1, "nt_store": 1,
                                      "grid_per_cu": 0, "tile_elems": 4096}, batched=True)
    assert ts.get_kernel_cfg("copy", "f64", 1 << 30, batched=True)["grid_per_cu"] == 0
    ts.set_kernel_cfg("copy", "f64", None, batched=True)


def test_candidate_sets_are_valid(ts):
    plain = ts.candidates()
    batched = ts.candidates(batched=True)
    assert len(plain) > 100 and len(batched) > 50
    keys = {tuple(sorted(c.items())) for c in plain}
    assert len(keys) == len(plain)
    for c in plain:
        ts.set_kernel_cfg("copy", "f64", c)
    for c in batched:
        ts.set_kernel_cfg("copy", "f64", c, batched=True)
        assert c["tile_elems"] % 8 == 0
    assert {c["tiles_per_wg"] for c in batched} == {1, 2, 4, 8}
    assert all(c["unroll"] <= 2 for c in batched if c["tiles_per_wg"] > 1)
    assert {c["record_ahead"] for c in batched} == {0, 1} and {c["record_ahead"] for c in plain} == {0}
    assert all(c["grid_per_cu"] == 0 and c["tiles_per_wg"] == 1 for c in batched if c["record_ahead"])
    assert {c["vec_bytes"] for c in batched} == {16, 8}
    assert all(c["wgs_per_tile"] == 1 for c in plain)
    pieces = [c for c in batched if c["wgs_per_tile"] > 1]
    assert pieces and all(c["block"] == 64 and c["unroll"] == 1 and c["record_ahead"] == 0 for c in pieces)
    assert all(c["vec_bytes"] == 16 for c in batched if c["wgs_per_tile"] == 1)
    ts.set_kernel_cfg("copy", "f64", None)
    ts.set_kernel_cfg("copy", "f64", None, batched=True)


# ------------------------------------------------- GPU-free planning rules
@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = tmp_path_factory.mktemp("shim") / "layout_shim.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-shared", "-fPIC", "-Wall", "-I" + CSRC, "-o", str(out),
                    os.path.join(ROOT, "tests", "cpp", "layout_shim.cpp")], check=True)
    lib = ctypes.CDLL(str(out))
    U = ctypes.POINTER(ctypes.c_uint64)
    lib.shim_check_map.argtypes = [ctypes.c_int, ctypes.c_int, U, U, U, U]
    lib.shim_align_class.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.shim_plan_plain.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, U]
    lib.shim_plan_batch.argtypes = [U, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int64, U, ctypes.c_size_t,
                                    U, U, U]
    lib.shim_check_batch_overlap.argtypes = [U, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_char_p,
                                             ctypes.c_size_t]
    lib.shim_cap_grid.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.shim_cap_grid.restype = ctypes.c_uint64
    return lib


def test_grids_stay_below_the_lane_count_limit(shim):
    """A launch's lanes (grid x block) are counted in 32 bits and its grid.x
    in 31: grid-stride launches are capped below both, and grids within them
    are left alone."""
    lanes, gx = (1 << 32) - 1, (1 << 31) - 1
    for block in (64, 128, 256, 512, 1024):
        for grid in (1, 1000, lanes // block, lanes // block + 1, (1 << 26) + 1, 1 << 40):
            g = shim.shim_cap_grid(grid, block)
            assert g * block <= lanes and g <= gx
            assert g == min(grid, lanes // block, gx)
    # the one-wave binary64 triad at 2^32 + 9 elements: one pass would need 2^32 + 64 lanes
    assert shim.shim_cap_grid(((1 << 32) + 9 + 63) // 64, 64) == lanes // 64


def _u64(vals):
    return (ctypes.c_uint64 * len(vals))(*vals)


def check_map(shim, uses_y, dev, x, y, d):
    cnt = ctypes.c_uint64()
    st = shim.shim_check_map(uses_y, dev, _u64(x), _u64(y), _u64(d), ctypes.byref(cnt))
    return st, cnt.value


def test_check_map_rules(shim):
    B = 1 << 20
    x = [B, 100, 0, 0]
    y = [2 * B, 100, 0, 0]
    d = [3 * B, 100, 0, 0]
    assert check_map(shim, 1, 0, x, y, d) == (TS_OK, 100)
    assert check_map(shim, 1, 0, x, y, [3 * B, 99, 0, 0])[0] == TS_E_SHAPE
    assert check_map(shim, 1, 0, x, [2 * B, 99, 0, 0], d)[0] == TS_E_SHAPE
    assert check_map(shim, 0, 0, x, [2 * B, 5, 1, 3], d) == (TS_OK, 100)  # y unused by copy/scale
    assert check_map(shim, 1, 0, x, [2 * B, 100, 1, 0], d)[0] == TS_E_DTYPE
    assert check_map(shim, 1, 0, x, y, [3 * B, 100, 2, 0])[0] == TS_E_DTYPE
    assert check_map(shim, 1, 1, x, y, d)[0] == TS_E_PLACEMENT
    assert check_map(shim, 1, 0, x, y, [3 * B, 100, 0, 1])[0] == TS_E_PLACEMENT
    assert check_map(shim, 1, 0, x, y, [B, 100, 0, 0]) == (TS_OK, 100)            # in place on x
    assert check_map(shim, 1, 0, x, y, [2 * B, 100, 0, 0]) == (TS_OK, 100)        # in place on y
    assert check_map(shim, 1, 0, x, y, [B + 8, 100, 0, 0])[0] == TS_E_ALIAS       # partial overlap
    assert check_map(shim, 1, 0, x, y, [B - 8 * 99, 100, 0, 0])[0] == TS_E_ALIAS
    assert check_map(shim, 1, 0, x, y, [B - 8 * 100, 100, 0, 0]) == (TS_OK, 100)  # adjacent, disjoint
    assert check_map(shim, 1, 0, [B, 0, 0, 0], y, [B + 8, 0, 0, 0]) == (TS_OK, 0)
    # inputs may overlap each other (read-only)
    assert check_map(shim, 1, 0, x, [B + 8, 100, 0, 0], d) == (TS_OK, 100)


def test_align_class(shim):
    assert shim.shim_align_class(256, 1, 512, 1024) == 0
    assert shim.shim_align_class(264, 1, 520, 1032) == 1
    assert shim.shim_align_class(264, 0, 0, 1032) == 1
    assert shim.shim_align_class(264, 1, 512, 1032) == 2
    assert shim.shim_align_class(256, 1, 512, 1028) == 2


@pytest.mark.parametrize("es,vb", [(8, 16), (8, 8), (4, 16), (4, 8), (4, 4), (2, 16), (2, 8), (2, 2)])
def test_plan_plain_partitions_the_range(shim, es, vb):
    rng = np.random.default_rng(es * 100 + vb)
    out = _u64([0, 0, 0])
    for _ in range(300):
        count = int(rng.integers(0, 200))
        mis = int(rng.integers(0, 16 // es)) * es
        base = 1 << 16
        ok = shim.shim_plan_plain(base + mis, 1, 2 * base + mis, 3 * base + mis, count, es, vb, out)
        assert ok == 1
        head, nvec, tail = out[0], out[1], out[2]
        assert head + nvec * (vb // es) + tail == count
        if nvec:
            # all three share the misalignment: the body starts on a 128-byte line
            assert (3 * base + mis + head * es) % 128 == 0
        assert tail < vb // es and head < 128 // es
    # shared misalignment modulo vb but not modulo 128: peel only to vb
    if vb > es:
        assert shim.shim_plan_plain(1 << 16, 1, (1 << 17) + 16, 1 << 18, 1000, es, vb, out) == 1
        assert out[0] == 0 and out[1] == 1000 // (vb // es)
    # different misalignments cannot share a vector body
    if vb > es:
        assert shim.shim_plan_plain(1 << 16, 1, (1 << 17) + es, 1 << 18, 100, es, vb, out) == 0


def plan_batch(shim, descs, es, tile):
    flat = [v for d in descs for v in d]
    cap = 100000
    tiles = (ctypes.c_uint64 * (3 * cap))()
    meta = (ctypes.c_uint64 * (2 * max(1, len(descs))))()
    nt, tot = ctypes.c_uint64(), ctypes.c_uint64()
    st = shim.shim_plan_batch(_u64(flat or [0]), len(descs), es, tile, tiles, cap, meta, ctypes.byref(nt),
                              ctypes.byref(tot))
    if st != 0:
        return st, None, None, None
    t = np.frombuffer(tiles, np.uint64, 3 * nt.value).reshape(-1, 3)
    m = np.frombuffer(meta, np.uint64, 2 * len(descs)).reshape(-1, 2)
    return st, t, m, tot.value


@pytest.mark.parametrize("es", [8, 4, 2])
@pytest.mark.parametrize("tile", [8, 64, 1024])
def test_plan_batch_covers_every_element_once(shim, es, tile):
    rng = np.random.default_rng(es + tile)
    descs = []
    base = 1 << 30
    for i in range(60):
        n = int(rng.choice([0, 1, 2, 3, 7, 8, 9, int(rng.integers(10, 5000))]))
        mis = [int(rng.integers(0, 16 // es)) * es for _ in range(3)]
        if i % 3:
            mis = [mis[0]] * 3
        descs.append([base + mis[0], base + (1 << 24) + mis[1], base + (2 << 24) + mis[2], n])
        base += 3 << 24
    st, t, m, total = plan_batch(shim, descs, es, tile)
    assert st == 0
    assert total == sum(d[3] for d in descs)
    for i, d in enumerate(descs):
        mine = t[t[:, 0] == i]
        n = d[3]
        if n == 0:
            assert mine.size == 0
            continue
        # consecutive, covering [0, n) exactly once
        assert mine[0, 1] == 0 and mine[-1, 2] == n
        assert np.all(mine[1:, 1] == mine[:-1, 2]) and np.all(mine[:, 2] > mine[:, 1])
        head, vec_ok = int(m[i, 0]), int(m[i, 1])
        shared = len({(x % 16) for x in d[:3]}) == 1
        assert vec_ok == int(shared)
        if vec_ok:
            assert (d[2] + head * es) % 16 == 0 and head < 16 // es
            # inner boundaries sit at head + k * tile
            for s in mine[1:, 1]:
                assert (int(s) - min(head, n)) % tile == 0
        assert np.all(mine[:, 2] - mine[:, 1] <= tile + head)
    # tiles of one instance are consecutive in the table, instances in order
    assert np.all(np.diff(t[:, 0].astype(np.int64)) >= 0)


def test_plan_batch_rejects_bad_input(shim):
    assert plan_batch(shim, [[0, 0, 0, 5]], 8, 64)[0] == TS_E_INVALID           # NULL arrays
    assert plan_batch(shim, [[1 << 20, 1 << 21, (1 << 22) + 4, 5]], 8, 64)[0] == TS_E_INVALID  # misaligned
    assert plan_batch(shim, [[1 << 20, 1 << 21, 1 << 22, 5]], 8, 60)[0] == TS_E_INVALID        # tile % 8
    assert plan_batch(shim, [[0, 0, 0, 0]], 8, 64)[0] == 0                      # empty instance is fine


@pytest.mark.parametrize("cmd", [
    ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-x", "c"],
    ["g++", "-std=c++11", "-pedantic", "-Wall", "-Wextra", "-Werror", "-x", "c++"],
])
def test_header_is_plain_c_and_cxx(cmd, tmp_path):
    """include/tstream.h compiles on its own as strict C99 and C++11."""
    src = tmp_path / "inc.c"
    src.write_text('#include "tstream.h"\nint main(void) { return ts_version(0, 0) == 0 ? 0 : 1; }\n')
    subprocess.run(cmd + ["-fsyntax-only", "-I" + os.path.join(ROOT, "include"), str(src)], check=True)


def test_c_client_on_a_host_target(tmp_path):
    """The plain C consumer of the ABI, built against the header and the
    library alone, runs its host-target mode: STREAM with the closed form,
    a run-time-compiled transform, and GPU-only calls refused."""
    out = tmp_path / "stream_client"
    lib_dir = os.path.join(ROOT, "paper_2206_06302_amd")
    subprocess.run(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-ffp-contract=off",
                    "-I" + os.path.join(ROOT, "include"), "-o", str(out),
                    os.path.join(ROOT, "tests", "cpp", "stream_client.c"), "-L" + lib_dir, "-ltstream",
                    "-Wl,-rpath," + lib_dir], check=True)
    r = subprocess.run([str(out), "100003", "host"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout and r.stdout.count("ok  ") == 6


# ------------------------------------------------------- batch overlap rule
def batch_overlap(shim, descs, es):
    flat = [v for d in descs for v in d]
    msg = ctypes.create_string_buffer(256)
    st = shim.shim_check_batch_overlap(_u64(flat or [0]), len(descs), es, msg, 256)
    return st, msg.value.decode()


def _brute_overlap(descs, es):
    """Reference: every pair of distinct arrays, within one instance
    (identical pointers allowed) or across instances (any shared byte)."""
    arrs = []
    for i, (a, b, c, n) in enumerate(descs):
        if n == 0:
            continue
        seen = set()
        for p in (a, b, c):
            if p in seen:
                continue
            seen.add(p)
            arrs.append((p, p + n * es, i))
    for k in range(len(arrs)):
        for m in range(k + 1, len(arrs)):
            (lo1, hi1, _), (lo2, hi2, _) = arrs[k], arrs[m]
            if lo1 < hi2 and lo2 < hi1:
                return TS_E_ALIAS
    return TS_OK


def test_batch_overlap_rules(shim):
    B = 1 << 30
    n = 1000
    ok = [[B, B + 8 * n, B + 16 * n, n], [B + 24 * n, B + 32 * n, B + 40 * n, n]]
    assert batch_overlap(shim, ok, 8) == (TS_OK, "")
    # in place inside one instance: the very same array is allowed
    assert batch_overlap(shim, [[B, B, B + 8 * n, n]], 8)[0] == TS_OK
    assert batch_overlap(shim, [[B, B, B, n]], 8)[0] == TS_OK
    # partial overlap inside one instance
    st, msg = batch_overlap(shim, [[B, B + 8, B + 16 * n, n]], 8)
    assert st == TS_E_ALIAS and "instance 0" in msg and "partly overlap" in msg
    # two instances sharing an array, identical or shifted
    st, msg = batch_overlap(shim, [ok[0], [B, B + 48 * n, B + 56 * n, n]], 8)
    assert st == TS_E_ALIAS and "instances 0 and 1" in msg
    st, msg = batch_overlap(shim, [ok[0], [B + 16 * n + 8 * (n - 1), B + 48 * n, B + 56 * n, n]], 8)
    assert st == TS_E_ALIAS
    # adjacent arrays share no byte
    assert batch_overlap(shim, [ok[0], [B + 24 * n, B + 32 * n, B + 40 * n, n]], 8)[0] == TS_OK
    # zero-length instances hold no memory
    assert batch_overlap(shim, [ok[0], [B, B, B, 0]], 8)[0] == TS_OK
    # a range past the end of the address space
    assert batch_overlap(shim, [[2 ** 64 - 64, B, B + 8 * n, 16]], 8)[0] == TS_E_SHAPE
    assert batch_overlap(shim, [], 8)[0] == TS_OK


@pytest.mark.parametrize("es", [8, 2])
def test_batch_overlap_matches_brute_force(shim, es):
    rng = np.random.default_rng(es)
    for _ in range(400):
        count = int(rng.integers(1, 7))
        descs = []
        for _ in range(count):
            n = int(rng.choice([0, 1, 5, 40]))
            ptrs = [int(rng.integers(0, 64)) * es * 8 for _ in range(3)]
            if rng.random() < 0.3:
                ptrs[1] = ptrs[0]
            descs.append(ptrs + [n])
        assert batch_overlap(shim, descs, es)[0] == _brute_overlap(descs, es), descs
