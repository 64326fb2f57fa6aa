// capi_batch.cpp -- batched ragged instances and HIP graphs in the C ABI.
//
// A batch is many (a, b, c, len, q) instances executed by one launch per map
// (bulk execution over all instances, Sections 3.3 and 4.2): the host splits
// every instance into tiles and uploads a table of self-contained tile
// records; each map reads the table of its configuration's tile size.
// Graphs capture one or more four-map iterations for replay.
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "capi_internal.hpp"

using namespace ts;
using namespace tsapi;

namespace tsapi {

void bump_epoch(ts_batch_s* b) {
  if (b->plan_epoch) ++*b->plan_epoch;
}

// Copy a tile table to a new device allocation (blocking).  On failure
// nothing is left allocated.
int upload_tiles(ts_target_s* t, const std::vector<BatchTile>& tiles, BatchTile** out) {
  *out = nullptr;
  if (tiles.empty()) return TS_OK;
  BatchTile* d = nullptr;
  TS_HIP(hipMalloc(&d, tiles.size() * sizeof(BatchTile)));
  hipError_t e =
      hipMemcpyAsync(d, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice, t->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "tile table upload");
  }
  *out = d;
  return TS_OK;
}

// Plan the batch's primary tiles with tile_elems and upload them (blocking).
// The old plan stays in place, whole, until the new one is on the device;
// on failure the batch is unchanged.
int batch_replan(ts_batch_s* b, int64_t tile_elems) {
  std::string err;
  std::vector<BatchDesc> descs;
  std::vector<BatchTile> tiles;
  uint64_t total = 0;
  int st = plan_batch(b->host.data(), b->host.size(), dtype_size(b->dtype), tile_elems, descs, tiles, total,
                      err);
  if (st != ST_OK) return fail(st, "%s", err.c_str());
  if (!b->d_expected && !descs.empty()) {
    TS_HIP(hipMalloc(&b->d_expected, descs.size() * sizeof(double)));
    TS_HIP(hipMalloc(&b->d_counts, descs.size() * sizeof(unsigned long long)));
    TS_HIP(hipHostMalloc(&b->h_expected, descs.size() * sizeof(double), hipHostMallocDefault));
    TS_HIP(hipHostMalloc(&b->h_counts, descs.size() * sizeof(unsigned long long), hipHostMallocDefault));
  }
  BatchTile* d_new = nullptr;
  if ((st = upload_tiles(b->target, tiles, &d_new)) != TS_OK) return st;
  if (b->d_tiles) {
    bump_epoch(b);
    // Maps of this batch may run on any stream of the device (every target
    // of it may execute the batch): none may still read the old table.
    (void)hipDeviceSynchronize();
    (void)hipFree(b->d_tiles);
  }
  b->d_tiles = d_new;
  b->descs.swap(descs);
  b->tiles.swap(tiles);
  b->total = total;
  b->tile_elems = tile_elems;
  return TS_OK;
}

void free_op_plans(ts_batch_s* b) {
  if (b->op_plans.empty()) return;
  bump_epoch(b);
  (void)hipDeviceSynchronize();  // as in batch_replan: no launch may still read these tables
  for (const ts_batch_s::OpPlan& p : b->op_plans)
    if (p.d_tiles) (void)hipFree(p.d_tiles);
  b->op_plans.clear();
}

ts_kernel_cfg batch_cfg(const ts_batch_s* b, int op) {
  const ts_kernel_cfg c = tune_table().lookup(op, b->dtype, b->total, TS_ALIGN_16, 1);
  log_choice(op, b->dtype, b->total, TS_ALIGN_16, 1, c);
  return c;
}

// Plans for the tile sizes of the four maps' configurations that differ from
// the primary plan's (blocking).  Nothing is planned when the tile is pinned.
int build_op_plans(ts_batch_s* b) {
  free_op_plans(b);
  if (b->tile_pinned || b->tiles.empty()) return TS_OK;
  for (int op = TS_COPY; op <= TS_TRIAD; ++op) {
    const int64_t tile = batch_cfg(b, op).tile_elems;
    if (tile <= 0 || tile == b->tile_elems) continue;
    bool have = false;
    for (const ts_batch_s::OpPlan& p : b->op_plans) have = have || p.tile_elems == tile;
    if (have) continue;
    std::string err;
    std::vector<BatchDesc> descs;
    std::vector<BatchTile> tiles;
    uint64_t total = 0;
    const int st = plan_batch(b->host.data(), b->host.size(), dtype_size(b->dtype), tile, descs, tiles,
                              total, err);
    if (st != ST_OK) return fail(st, "%s", err.c_str());
    ts_batch_s::OpPlan p{tile, tiles.size(), nullptr};
    const int ust = upload_tiles(b->target, tiles, &p.d_tiles);
    if (ust != TS_OK) return ust;
    b->op_plans.push_back(p);
  }
  return TS_OK;
}

int launch_batch(ts_target_s* t, ts_batch_s* b, int op, const ts_kernel_cfg& cfg) {
  if (b->tiles.empty()) return TS_OK;
  BatchLaunch L{};
  L.tiles = b->d_tiles;
  L.ntiles = b->tiles.size();
  if (!b->tile_pinned && cfg.tile_elems > 0 && cfg.tile_elems != b->tile_elems) {
    for (const ts_batch_s::OpPlan& p : b->op_plans)
      if (p.tile_elems == cfg.tile_elems) {
        L.tiles = p.d_tiles;
        L.ntiles = p.ntiles;
      }
  }
  L.op = op;
  L.unroll = cfg.unroll;
  L.ntl = cfg.nt_load;
  L.nts = cfg.nt_store;
  L.stream = t->stream;
  if (cfg.wgs_per_tile > 1) {
    // One-wave workgroups that share each tile, one piece each; the kernel
    // strides over whatever lies beyond the largest launch.  Its first piece
    // is taken unchecked, so the grid is at least 1 and at most ntiles * P.
    if (L.ntiles == 0) return TS_OK;
    int lg = 0;
    while ((1 << lg) < cfg.wgs_per_tile) ++lg;
    const uint64_t grid = cap_grid(L.ntiles << lg, 64);
    L.grid = static_cast<uint32_t>(grid);
    L.block = 64;
    L.tiles_per_wg = 1;
    L.record_ahead = 0;
    L.pieces_log2 = lg;
    L.vb = cfg.vec_bytes;
    const hipError_t e = batch_launch(b->dtype, L);
    if (e != hipSuccess) return hip_fail(e, "batched STREAM kernel launch");
    return TS_OK;
  }
  // grid_per_cu 0: one workgroup per group of tiles_per_wg consecutive
  // tiles; otherwise a persistent grid that strides over the groups.
  const uint64_t per_wg = cfg.tiles_per_wg > 1 ? static_cast<uint64_t>(cfg.tiles_per_wg) : 1;
  const uint64_t groups = (L.ntiles + per_wg - 1) / per_wg;
  uint64_t grid = cfg.grid_per_cu > 0
                      ? static_cast<uint64_t>(cfg.grid_per_cu) * static_cast<uint64_t>(t->info.compute_units)
                      : groups;
  if (grid > groups) grid = groups;
  grid = cap_grid(grid, static_cast<uint64_t>(cfg.block));  // the kernel strides over the rest
  if (grid < 1) grid = 1;
  L.grid = static_cast<uint32_t>(grid);
  L.block = static_cast<uint32_t>(cfg.block);
  L.tiles_per_wg = static_cast<int>(per_wg);
  L.record_ahead = cfg.record_ahead && per_wg == 1 && grid >= L.ntiles ? 1 : 0;
  L.pieces_log2 = 0;
  L.vb = 16;
  const hipError_t e = batch_launch(b->dtype, L);
  if (e != hipSuccess) return hip_fail(e, "batched STREAM kernel launch");
  return TS_OK;
}

int check_batch_exec(ts_target_s* t, ts_batch_s* b) {
  if (!ok_target(t)) return fail(TS_E_INVALID, "invalid target handle");
  if (t->host) return host_only_gpu("batched execution");
  if (!ok_batch(b)) return fail(TS_E_INVALID, "invalid batch handle");
  if (b->device != t->device)
    return fail(TS_E_PLACEMENT, "batch is placed on device %d, the executor runs on device %d",
                b->device, t->device);
  return use_device(t->device);
}

// Fills and mismatch counts over a batch give each workgroup about 16 KiB of
// tiles: one tile of 16 KiB or more, else up to four consecutive ones.  With
// one per tile, the workgroups of 512-element (4 KiB) binary64 tiles are
// dispatched more slowly than they stream (mismatch count 4.7 against 5.5
// TB/s with four; uniform fill 3.9 against 4.1); with 2048-element tiles one
// per workgroup is the faster (constant fill 5.59-5.65 against 5.40-5.42
// TB/s with four, mismatch count 7.26-7.27 against 7.19).
uint32_t aux_tiles_per_wg(const ts_batch_s* b) {
  const uint64_t tile_bytes = static_cast<uint64_t>(b->tile_elems) * dtype_size(b->dtype);
  const uint64_t k = tile_bytes ? 16384 / tile_bytes : kAuxMaxTilesPerWg;
  return static_cast<uint32_t>(k < 1 ? 1 : (k > kAuxMaxTilesPerWg ? kAuxMaxTilesPerWg : k));
}

uint32_t aux_grid(uint64_t ntiles, uint32_t per_wg) {
  const uint64_t g = cap_grid((ntiles + per_wg - 1) / per_wg, kAuxBlock);
  return static_cast<uint32_t>(g < 1 ? 1 : g);
}

}  // namespace tsapi

extern "C" {

// ---------------------------------------------------------------------------
// Batched instances
// ---------------------------------------------------------------------------
int ts_batch_create(ts_target t, ts_dtype dtype, const ts_batch_desc* descs, size_t count,
                    ts_batch* out) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !out) return fail(TS_E_INVALID, "invalid target handle or NULL out");
  if (t->host) return host_only_gpu("batched execution");
  if (!valid_dtype(dtype)) return fail(TS_E_INVALID, "unknown dtype");
  if (!map_dtype(dtype)) return fail(TS_E_UNSUPPORTED, "batches take floating-point storage");
  if (count > 0 && !descs) return fail(TS_E_INVALID, "NULL descriptors");
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  ts_batch_s* b = new ts_batch_s();
  b->plan_epoch = std::make_shared<uint64_t>(0);
  b->target = t;
  b->device = t->device;
  b->dtype = dtype;
  b->host.resize(count);
  for (size_t i = 0; i < count; ++i) {
    const ts_batch_desc& d = descs[i];
    b->host[i] = HostDesc{reinterpret_cast<uintptr_t>(d.a), reinterpret_cast<uintptr_t>(d.b),
                          reinterpret_cast<uintptr_t>(d.c), d.len, d.q};
  }
  auto cleanup = [&](int status) {
    free_op_plans(b);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_expected) (void)hipFree(b->d_expected);
    if (b->d_counts) (void)hipFree(b->d_counts);
    if (b->h_expected) (void)hipHostFree(b->h_expected);
    if (b->h_counts) (void)hipHostFree(b->h_counts);
    delete b;
    return status;
  };
  // Placement: every array of every instance lies, whole, in one device
  // allocation of this device; then no two instances share memory, and the
  // arrays of one instance are identical or disjoint.
  const size_t es = dtype_size(dtype);
  for (size_t i = 0; i < count; ++i) {
    if (descs[i].len == 0) continue;
    const void* arrs[3] = {descs[i].a, descs[i].b, descs[i].c};
    for (int w = 0; w < 3; ++w) {
      if (!arrs[w]) return cleanup(fail(TS_E_INVALID, "instance %zu: NULL array with len > 0", i));
      char what[64];
      std::snprintf(what, sizeof what, "instance %zu array %c", i, "abc"[w]);
      const int rs = check_device_range(t->device, arrs[w], descs[i].len, es, what);
      if (rs != TS_OK) return cleanup(rs);
    }
  }
  {
    std::string err;
    const int os = check_batch_overlap(b->host.data(), b->host.size(), es, err);
    if (os != ST_OK) return cleanup(fail(os, "%s", err.c_str()));
  }
  const ts_kernel_cfg cfg = tune_table().lookup(TS_TRIAD, dtype, 0, TS_ALIGN_16, 1);
  uint64_t total = 0;
  for (size_t i = 0; i < count; ++i) total += descs[i].len;
  const ts_kernel_cfg sized = tune_table().lookup(TS_TRIAD, dtype, total, TS_ALIGN_16, 1);
  int64_t tile = sized.tile_elems > 0 ? sized.tile_elems : (cfg.tile_elems > 0 ? cfg.tile_elems : 16384);
  st = batch_replan(b, tile);
  if (st == TS_OK) st = build_op_plans(b);
  if (st != TS_OK) return cleanup(st);
  b->magic = kBatchMagic;
  *out = b;
  return TS_OK;
  TS_GUARD_END
}

int ts_batch_destroy(ts_batch b) {
  if (!b) return TS_OK;
  if (!ok_batch(b)) return fail(TS_E_INVALID, "invalid batch handle");
  (void)use_device(b->device);
  (void)hipDeviceSynchronize();  // the batch's maps may run on any stream of its device
  free_op_plans(b);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_expected) (void)hipFree(b->d_expected);
  if (b->d_counts) (void)hipFree(b->d_counts);
  if (b->h_expected) (void)hipHostFree(b->h_expected);
  if (b->h_counts) (void)hipHostFree(b->h_counts);
  *b->plan_epoch = kDeadEpoch;
  b->magic = kDead;
  delete b;
  return TS_OK;
}

int ts_batch_info(ts_batch b, size_t* count, uint64_t* total, uint64_t* tiles, int64_t* tile_elems) {
  if (!ok_batch(b)) return fail(TS_E_INVALID, "invalid batch handle");
  if (count) *count = b->host.size();
  if (total) *total = b->total;
  if (tiles) *tiles = b->tiles.size();
  if (tile_elems) *tile_elems = b->tile_elems;
  return TS_OK;
}

int ts_batch_set_tile(ts_batch b, int64_t tile_elems) {
  TS_GUARD_BEGIN
  if (!ok_batch(b) || !ok_target(b->target)) return fail(TS_E_INVALID, "invalid batch handle");
  int st = use_device(b->device);
  if (st != TS_OK) return st;
  if ((st = batch_replan(b, tile_elems)) != TS_OK) return st;
  b->tile_pinned = true;
  free_op_plans(b);
  return TS_OK;
  TS_GUARD_END
}

int ts_batch_op(ts_target exec, ts_batch b, ts_op op) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(exec, b);
  if (st != TS_OK) return st;
  if (!valid_op(op)) return fail(TS_E_INVALID, "bad op");
  return launch_batch(exec, b, op, batch_cfg(b, op));
  TS_GUARD_END
}

int ts_batch_op_plain(ts_target exec, ts_batch b, ts_op op) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(exec, b);
  if (st != TS_OK) return st;
  if (!valid_op(op)) return fail(TS_E_INVALID, "bad op");
  for (const HostDesc& h : b->host) {
    if (h.len == 0) continue;
    const void* x;
    const void* y = nullptr;
    void* d;
    switch (op) {  // Listing 4 roles inside every instance
      case TS_COPY: x = reinterpret_cast<void*>(h.a); d = reinterpret_cast<void*>(h.c); break;
      case TS_SCALE: x = reinterpret_cast<void*>(h.c); d = reinterpret_cast<void*>(h.b); break;
      case TS_ADD: x = reinterpret_cast<void*>(h.a); y = reinterpret_cast<void*>(h.b); d = reinterpret_cast<void*>(h.c); break;
      default: x = reinterpret_cast<void*>(h.b); y = reinterpret_cast<void*>(h.c); d = reinterpret_cast<void*>(h.a); break;
    }
    const uintptr_t ya = reinterpret_cast<uintptr_t>(y);
    const int cls = align_class(reinterpret_cast<uintptr_t>(x), y ? &ya : nullptr, reinterpret_cast<uintptr_t>(d));
    const ts_kernel_cfg cfg = tune_table().lookup(op, b->dtype, h.len, cls, 0);
    if ((st = launch_map(exec, op, b->dtype, x, y, d, h.len, h.q, cfg)) != TS_OK) return st;
  }
  return TS_OK;
  TS_GUARD_END
}

int ts_batch_fill(ts_target exec, ts_batch b, int which, double value) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(exec, b);
  if (st != TS_OK) return st;
  if (which < 0 || which > 2) return fail(TS_E_INVALID, "which must be 0 (a), 1 (b) or 2 (c)");
  if (b->tiles.empty()) return TS_OK;
  const uint32_t per_wg = aux_tiles_per_wg(b);
  const hipError_t e = launch_batch_fill(b->dtype, b->d_tiles, b->tiles.size(), per_wg, which, 0, value, 0,
                                         aux_grid(b->tiles.size(), per_wg), exec->stream);
  if (e != hipSuccess) return hip_fail(e, "batched fill launch");
  return TS_OK;
  TS_GUARD_END
}

int ts_batch_fill_uniform(ts_target exec, ts_batch b, int which, uint64_t seed) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(exec, b);
  if (st != TS_OK) return st;
  if (which < 0 || which > 2) return fail(TS_E_INVALID, "which must be 0 (a), 1 (b) or 2 (c)");
  if (b->host.size() > (((1ull << 16) - 16) / 3))
    return fail(TS_E_UNSUPPORTED, "too many instances for 16-bit stream ids");
  if (b->tiles.empty()) return TS_OK;
  const uint32_t per_wg = aux_tiles_per_wg(b);
  const hipError_t e = launch_batch_fill(b->dtype, b->d_tiles, b->tiles.size(), per_wg, which, 1, 0.0, seed,
                                         aux_grid(b->tiles.size(), per_wg), exec->stream);
  if (e != hipSuccess) return hip_fail(e, "batched uniform fill launch");
  return TS_OK;
  TS_GUARD_END
}

int ts_batch_mismatch_count(ts_target exec, ts_batch b, int which, const double* expected,
                            uint64_t* counts) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(exec, b);
  if (st != TS_OK) return st;
  if (which < 0 || which > 2) return fail(TS_E_INVALID, "which must be 0 (a), 1 (b) or 2 (c)");
  const size_t n = b->host.size();
  if (n == 0) return TS_OK;
  if (!expected || !counts) return fail(TS_E_INVALID, "NULL expected or counts");
  // The staging buffers are free: every earlier call ended with a stream
  // synchronisation after its last copy.
  std::memcpy(b->h_expected, expected, n * sizeof(double));
  TS_HIP(hipMemcpyAsync(b->d_expected, b->h_expected, n * sizeof(double), hipMemcpyHostToDevice, exec->stream));
  hipError_t e = launch_zero_u64(b->d_counts, n, exec->stream);
  if (e != hipSuccess) return hip_fail(e, "zero kernel launch");
  if (!b->tiles.empty()) {
    const uint32_t per_wg = aux_tiles_per_wg(b);
    e = launch_batch_mismatch(b->dtype, b->d_tiles, b->tiles.size(), per_wg, which, b->d_expected, b->d_counts,
                              aux_grid(b->tiles.size(), per_wg), exec->stream);
    if (e != hipSuccess) return hip_fail(e, "batched mismatch launch");
  }
  TS_HIP(hipMemcpyAsync(b->h_counts, b->d_counts, n * sizeof(uint64_t), hipMemcpyDeviceToHost, exec->stream));
  TS_HIP(hipStreamSynchronize(exec->stream));
  std::memcpy(counts, b->h_counts, n * sizeof(uint64_t));
  return TS_OK;
  TS_GUARD_END
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Graphs
// ---------------------------------------------------------------------------
namespace {

template <class Body>
int capture(ts_target_s* t, Body&& body, ts_graph* out, const ts_batch_s* batch = nullptr) {
  if (!out) return fail(TS_E_INVALID, "NULL out");
  if (t->host) return host_only_gpu("graph capture");
  if (t->stream == nullptr)
    return fail(TS_E_UNSUPPORTED, "graph capture needs a target with a non-default stream");
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  TS_HIP(hipStreamBeginCapture(t->stream, hipStreamCaptureModeThreadLocal));
  st = body();
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(t->stream, &graph);
  if (st != TS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(ie, "hipGraphInstantiate");
  }
  ts_graph_s* g = new ts_graph_s();
  g->device = t->device;
  g->graph = graph;
  g->exec = exec;
  if (batch) {
    g->batch_epoch = batch->plan_epoch;
    g->epoch_at_capture = *batch->plan_epoch;
  }
  g->magic = kGraphMagic;
  *out = g;
  return TS_OK;
}

}  // namespace

extern "C" {

int ts_graph_capture_stream_iterations(ts_target t, ts_batch b, int iterations, ts_graph* out) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(t, b);
  if (st != TS_OK) return st;
  if (iterations < 1 || iterations > TS_GRAPH_MAX_ITERATIONS)
    return fail(TS_E_INVALID, "iterations must be in [1, TS_GRAPH_MAX_ITERATIONS]");
  return capture(
      t,
      [&]() {
        for (int k = 0; k < iterations; ++k)
          for (int op = TS_COPY; op <= TS_TRIAD; ++op) {
            const int s = launch_batch(t, b, op, batch_cfg(b, op));
            if (s != TS_OK) return s;
          }
        return static_cast<int>(TS_OK);
      },
      out, b);
  TS_GUARD_END
}

int ts_graph_capture_stream_iteration(ts_target t, ts_batch b, ts_graph* out) {
  return ts_graph_capture_stream_iterations(t, b, 1, out);
}

int ts_graph_capture_batch_op(ts_target t, ts_batch b, ts_op op, ts_graph* out) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(t, b);
  if (st != TS_OK) return st;
  if (!valid_op(op)) return fail(TS_E_INVALID, "bad op");
  return capture(t, [&]() { return launch_batch(t, b, op, batch_cfg(b, op)); }, out, b);
  TS_GUARD_END
}

int ts_graph_capture_arrays_iterations(ts_target t, ts_array a, ts_array b, ts_array c, double q,
                                       int iterations, ts_graph* out) {
  TS_GUARD_BEGIN
  if (!ok_target(t)) return fail(TS_E_INVALID, "invalid target handle");
  if (t->host) return host_only_gpu("graph capture");
  if (iterations < 1 || iterations > TS_GRAPH_MAX_ITERATIONS)
    return fail(TS_E_INVALID, "iterations must be in [1, TS_GRAPH_MAX_ITERATIONS]");
  const int st = capture(
      t,
      [&]() {
        for (int k = 0; k < iterations; ++k) {
          const int s = ts_stream_iteration(t, a, b, c, q);
          if (s != TS_OK) return s;
        }
        return static_cast<int>(TS_OK);
      },
      out);
  if (st == TS_OK) (*out)->arrays_alive = {a->alive, b->alive, c->alive};
  return st;
  TS_GUARD_END
}

int ts_graph_capture_arrays_iteration(ts_target t, ts_array a, ts_array b, ts_array c, double q,
                                      ts_graph* out) {
  return ts_graph_capture_arrays_iterations(t, a, b, c, q, 1, out);
}

int ts_graph_launch(ts_target t, ts_graph g, int repeats) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !ok_graph(g)) return fail(TS_E_INVALID, "invalid target or graph handle");
  if (t->host) return host_only_gpu("graph launch");
  if (repeats < 0) return fail(TS_E_INVALID, "negative repeat count");
  if (g->device != t->device) return fail(TS_E_PLACEMENT, "graph belongs to another device");
  if (g->batch_epoch && *g->batch_epoch != g->epoch_at_capture)
    return fail(TS_E_INVALID, "the graph's batch was re-planned or destroyed after capture");
  for (const std::shared_ptr<bool>& alive : g->arrays_alive)
    if (!*alive) return fail(TS_E_INVALID, "an array of the graph was freed after capture");
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  for (int r = 0; r < repeats; ++r) TS_HIP(hipGraphLaunch(g->exec, t->stream));
  return TS_OK;
  TS_GUARD_END
}

int ts_graph_destroy(ts_graph g) {
  if (!g) return TS_OK;
  if (!ok_graph(g)) return fail(TS_E_INVALID, "invalid graph handle");
  (void)use_device(g->device);
  (void)hipDeviceSynchronize();  // launches of it may still run on any stream of the device
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  g->magic = kDead;
  delete g;
  return TS_OK;
}

}  // extern "C"
