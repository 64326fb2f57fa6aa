// capi.cpp -- the C ABI of libtstream (declared in include/tstream.h).
//
// Targets pair a device with a stream (Sections 3.1 and 4.2); arrays are
// placed on a target's device and bulk-constructed there (Section 3.2);
// each algorithm call is one bulk launch on the executing target's stream
// (Sections 3.3 and 3.4).  Every entry point catches everything, returns a
// status and leaves a thread-local message on failure.
#include <hip/hip_runtime_api.h>

#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tstream.h"
#include "host_target.hpp"
#include "ts_handles.hpp"
#include "ts_internal.hpp"
#include "tune.hpp"

namespace {

// Largest grid.x of a launch; kernels stride over whatever lies beyond it.
constexpr uint64_t kMaxGridX = 0x7fffffffull;

using namespace ts;

thread_local std::string g_error;

int fail(int status, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();  // clear the sticky per-thread error state
  const int st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? TS_E_OOM : TS_E_DEVICE;
  return fail(st, "%s failed: %s (%d)", what, hipGetErrorString(e), static_cast<int>(e));
}

#define TS_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

#define TS_GUARD_BEGIN try {
#define TS_GUARD_END                                               \
  }                                                                \
  catch (const std::bad_alloc&) {                                  \
    return fail(TS_E_OOM, "host allocation failed");               \
  }                                                                \
  catch (const std::exception& ex) {                               \
    return fail(TS_E_INVALID, "internal error: %s", ex.what());    \
  }                                                                \
  catch (...) {                                                    \
    return fail(TS_E_INVALID, "internal error");                   \
  }

constexpr uint32_t kBatchMagic = 0x42415431u;
constexpr uint32_t kGraphMagic = 0x47524631u;
constexpr uint32_t kEventMagic = 0x45564e31u;
constexpr uint32_t kFutureMagic = 0x46555431u;
constexpr uint32_t kDead = 0xdeadbeefu;
constexpr uint64_t kDeadEpoch = ~0ull;
constexpr double kPeakBytesPerS = 8.0e12;  // MI355X HBM3E, the % of peak denominator

}  // namespace

namespace ts {
int api_fail(int status, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return status;
}
int api_hip_fail(hipError_t e, const char* what) { return hip_fail(e, what); }
}  // namespace ts

struct ts_batch_s {
  uint32_t magic;
  ts_target_s* target;
  int device;
  int dtype;
  std::vector<HostDesc> host;
  std::vector<BatchDesc> descs;  // host-side metadata (alignment per instance)
  std::vector<BatchTile> tiles;  // primary plan: fills, mismatch counts, info
  BatchTile* d_tiles;
  double* d_expected;
  unsigned long long* d_counts;
  uint64_t total;
  int64_t tile_elems;
  // Device plans for the other tile sizes that the maps' tuned configurations
  // ask for, so that each map runs on its own tiles.
  struct OpPlan {
    int64_t tile_elems;
    uint64_t ntiles;
    BatchTile* d_tiles;
  };
  std::vector<OpPlan> op_plans;
  bool tile_pinned;  // set by ts_batch_set_tile: every map uses the primary plan
  // Bumped whenever a tile table is freed (re-plan) and set to kDeadEpoch on
  // destruction; graphs captured from the batch share it and refuse to launch
  // once it has moved, instead of reading freed tile tables.
  std::shared_ptr<uint64_t> plan_epoch;
};

struct ts_graph_s {
  uint32_t magic;
  int device;
  hipGraph_t graph;
  hipGraphExec_t exec;
  std::shared_ptr<uint64_t> batch_epoch;  // null for graphs of plain arrays
  uint64_t epoch_at_capture;
};

struct ts_event_s {
  uint32_t magic;
  int device;
  hipEvent_t ev;
  bool recorded;
};

struct ts_future_s {
  uint32_t magic;
  std::mutex mu;
  std::condition_variable cv;
  bool ready;
};

namespace {

bool ok_target(const ts_target_s* t) { return t && t->magic == kTargetMagic; }
bool ok_array(const ts_array_s* a) { return a && a->magic == kArrayMagic; }
bool ok_batch(const ts_batch_s* b) { return b && b->magic == kBatchMagic; }
bool ok_graph(const ts_graph_s* g) { return g && g->magic == kGraphMagic; }
bool ok_event(const ts_event_s* e) { return e && e->magic == kEventMagic; }
bool ok_future(const ts_future_s* f) { return f && f->magic == kFutureMagic; }

constexpr int kHostDevice = -1;

int host_only_gpu(const char* what) {
  return fail(TS_E_UNSUPPORTED, "%s needs a GPU target (this is a host-CPU target)", what);
}

// Run fn(lo, hi, w) on every worker of a host target over its block of n.
template <class F>
void host_blocks(ts_target_s* t, uint64_t n, F&& fn) {
  const int W = t->pool->size();
  t->pool->run([&](int w) {
    uint64_t lo, hi;
    HostPool::block(n, W, w, &lo, &hi);
    fn(lo, hi, w);
  });
}

// Stream callback that makes a future ready (runs on a runtime thread).
void future_ready_cb(void* p) {
  ts_future_s* f = static_cast<ts_future_s*>(p);
  {
    std::lock_guard<std::mutex> lk(f->mu);
    f->ready = true;
  }
  f->cv.notify_all();
}

// Make `device` current for the calling thread (cheap when it already is).
int use_device(int device) {
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur == device) return TS_OK;
  TS_HIP(hipSetDevice(device));
  return TS_OK;
}

// Storage types of arrays (bytes included) and of the STREAM maps.
bool valid_dtype(int dt) { return dt >= TS_F64 && dt <= TS_U8; }
bool map_dtype(int dt) { return dt >= TS_F64 && dt <= TS_F16; }
bool valid_op(int op) { return op >= TS_COPY && op <= TS_TRIAD; }

uint64_t stream_bytes(int op, uint64_t n, size_t es) {
  return (op == TS_ADD || op == TS_TRIAD ? 3ull : 2ull) * n * es;
}

std::once_flag g_env_cache_once;

void load_env_cache() {
  const char* p = std::getenv("TS_TUNE_CACHE");
  if (!p || !*p) return;
  std::string err;
  if (tune_table().load(p, &err) != 0)
    std::fprintf(stderr, "tstream: ignoring tuning file (%s); using defaults\n", err.c_str());
}

hipError_t plain_launch(int dtype, const PlainLaunch& L) {
  switch (dtype) {
    case TS_F64: return plain_launch_f64(L);
    case TS_F32: return plain_launch_f32(L);
    case TS_BF16: return plain_launch_bf16(L);
    case TS_F16: return plain_launch_f16(L);
    default: return hipErrorInvalidValue;
  }
}

hipError_t batch_launch(int dtype, const BatchLaunch& L) {
  switch (dtype) {
    case TS_F64: return batch_launch_f64(L);
    case TS_F32: return batch_launch_f32(L);
    case TS_BF16: return batch_launch_bf16(L);
    case TS_F16: return batch_launch_f16(L);
    default: return hipErrorInvalidValue;
  }
}

Operand operand_of(const ts_array_s* a) {
  return Operand{reinterpret_cast<uintptr_t>(a->ptr), a->n, a->dtype, a->device};
}

// Launch one map over `count` elements with configuration `cfg`.
int launch_map(ts_target_s* t, int op, int dtype, const void* x, const void* y, void* d,
               uint64_t count, double q, const ts_kernel_cfg& cfg) {
  if (count == 0) return TS_OK;
  const size_t es = dtype_size(dtype);
  const bool has_y = op == TS_ADD || op == TS_TRIAD;
  const uintptr_t xa = reinterpret_cast<uintptr_t>(x), da = reinterpret_cast<uintptr_t>(d);
  const uintptr_t ya = reinterpret_cast<uintptr_t>(y);
  PlainPlan plan{};
  size_t vb = cfg.vec_bytes > 0 ? static_cast<size_t>(cfg.vec_bytes) : es;
  if (vb < es || !plan_plain(xa, has_y ? &ya : nullptr, da, count, es, vb, plan)) {
    vb = es;  // element-wise path: always aligned
    plan_plain(xa, has_y ? &ya : nullptr, da, count, es, vb, plan);
  }
  const uint64_t block = static_cast<uint64_t>(cfg.block);
  const uint64_t per_wg = block * static_cast<uint64_t>(cfg.unroll);
  uint64_t grid = (plan.nvec + per_wg - 1) / per_wg;
  if (grid < 1) grid = 1;
  if (cfg.grid_per_cu > 0) {
    const uint64_t cap = static_cast<uint64_t>(cfg.grid_per_cu) * static_cast<uint64_t>(t->info.compute_units);
    if (grid > cap) grid = cap;
  }
  if (grid > kMaxGridX) grid = kMaxGridX;  // the loop strides over the rest
  PlainLaunch L{};
  L.x = x;
  L.y = has_y ? y : x;
  L.d = d;
  L.q = q;
  L.qf = static_cast<float>(q);
  L.head = plan.head;
  L.nvec = plan.nvec;
  L.tail = plan.tail;
  L.grid = static_cast<uint32_t>(grid);
  L.block = static_cast<uint32_t>(block);
  L.op = op;
  L.vb = static_cast<int>(vb);
  L.unroll = cfg.unroll;
  L.ntl = cfg.nt_load;
  L.nts = cfg.nt_store;
  L.stream = t->stream;
  const hipError_t e = plain_launch(dtype, L);
  if (e != hipSuccess) return hip_fail(e, "STREAM kernel launch");
  return TS_OK;
}

int check_exec_arrays(ts_target_s* t, int op, ts_array_s* x, ts_array_s* y, ts_array_s* d,
                      uint64_t* count) {
  if (!ok_target(t)) return fail(TS_E_INVALID, "invalid target handle");
  const bool has_y = op == TS_ADD || op == TS_TRIAD;
  if (!ok_array(x) || !ok_array(d) || (has_y && !ok_array(y)))
    return fail(TS_E_INVALID, "invalid array handle");
  const Operand ox = operand_of(x), od = operand_of(d);
  Operand oy{};
  if (has_y) oy = operand_of(y);
  MapCheck r = check_map(has_y, t->device, ox, has_y ? &oy : nullptr, od);
  if (r.status != ST_OK) return fail(r.status, "%s", r.msg.c_str());
  *count = r.count;
  return TS_OK;
}

int run_map(ts_target_s* t, int op, ts_array_s* x, ts_array_s* y, ts_array_s* d, double q) {
  uint64_t count = 0;
  int st = check_exec_arrays(t, op, x, y, d, &count);
  if (st != TS_OK) return st;
  if (!map_dtype(x->dtype)) return fail(TS_E_UNSUPPORTED, "the STREAM maps take floating-point storage");
  if (count == 0) return TS_OK;
  const bool has_y = op == TS_ADD || op == TS_TRIAD;
  if (t->host) {
    if (x->dtype == TS_F64) {
      const double* xp = static_cast<const double*>(x->ptr);
      const double* yp = has_y ? static_cast<const double*>(y->ptr) : nullptr;
      double* dp = static_cast<double*>(d->ptr);
      host_blocks(t, count, [&](uint64_t lo, uint64_t hi, int) { host_map_f64(op, xp, yp, dp, lo, hi, q); });
    } else if (x->dtype == TS_F32) {
      const float* xp = static_cast<const float*>(x->ptr);
      const float* yp = has_y ? static_cast<const float*>(y->ptr) : nullptr;
      float* dp = static_cast<float*>(d->ptr);
      const float qf = static_cast<float>(q);
      host_blocks(t, count, [&](uint64_t lo, uint64_t hi, int) { host_map_f32(op, xp, yp, dp, lo, hi, qf); });
    } else {
      return fail(TS_E_UNSUPPORTED, "host targets support binary64 and binary32 storage");
    }
    return TS_OK;
  }
  if ((st = use_device(t->device)) != TS_OK) return st;
  const uintptr_t ya = has_y ? reinterpret_cast<uintptr_t>(y->ptr) : 0;
  const int cls = align_class(reinterpret_cast<uintptr_t>(x->ptr), has_y ? &ya : nullptr,
                              reinterpret_cast<uintptr_t>(d->ptr));
  const ts_kernel_cfg cfg = tune_table().lookup(op, x->dtype, count, cls, 0);
  return launch_map(t, op, x->dtype, x->ptr, has_y ? y->ptr : nullptr, d->ptr, count, q, cfg);
}

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
  return tune_table().lookup(op, b->dtype, b->total, TS_ALIGN_16, 1);
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
  // grid_per_cu 0: one workgroup per tile; otherwise a persistent grid that
  // strides over the tiles.
  uint64_t grid = cfg.grid_per_cu > 0
                      ? static_cast<uint64_t>(cfg.grid_per_cu) * static_cast<uint64_t>(t->info.compute_units)
                      : L.ntiles;
  if (grid > L.ntiles) grid = L.ntiles;
  if (grid > kMaxGridX) grid = kMaxGridX;
  if (grid < 1) grid = 1;
  L.grid = static_cast<uint32_t>(grid);
  L.block = static_cast<uint32_t>(cfg.block);
  L.op = op;
  L.unroll = cfg.unroll;
  L.ntl = cfg.nt_load;
  L.nts = cfg.nt_store;
  L.stream = t->stream;
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

uint32_t aux_grid(const ts_target_s* t, uint64_t ntiles) {
  uint64_t g = 4ull * static_cast<uint64_t>(t->info.compute_units);
  if (g > ntiles) g = ntiles;
  return static_cast<uint32_t>(g < 1 ? 1 : g);
}

// Seconds per launch of one candidate: `inner` back-to-back launches between
// two events (so small, launch-bound sizes are timed as throughput), repeated
// `reps` times after a warm-up; the median of the repetitions is returned.
template <class Launch>
int time_candidate(ts_target_s* t, int reps, int inner, Launch&& launch, double* seconds) {
  if (reps < 1) reps = 1;
  if (inner < 1) inner = 1;
  std::vector<hipEvent_t> ev(2 * static_cast<size_t>(reps), nullptr);
  int st = TS_OK;
  for (auto& e : ev) {
    const hipError_t he = hipEventCreate(&e);
    if (he != hipSuccess) {
      st = hip_fail(he, "hipEventCreate");
      break;
    }
  }
  if (st == TS_OK) st = launch();  // warm-up
  for (int r = 0; r < reps && st == TS_OK; ++r) {
    hipError_t he = hipEventRecord(ev[2 * r], t->stream);
    if (he != hipSuccess) {
      st = hip_fail(he, "hipEventRecord");
      break;
    }
    for (int i = 0; i < inner && st == TS_OK; ++i) st = launch();
    if (st != TS_OK) break;
    he = hipEventRecord(ev[2 * r + 1], t->stream);
    if (he != hipSuccess) st = hip_fail(he, "hipEventRecord");
  }
  std::vector<float> ms;
  if (st == TS_OK) {
    const hipError_t he = hipStreamSynchronize(t->stream);
    if (he != hipSuccess) st = hip_fail(he, "hipStreamSynchronize");
  }
  for (int r = 0; r < reps && st == TS_OK; ++r) {
    float v = 0;
    const hipError_t he = hipEventElapsedTime(&v, ev[2 * r], ev[2 * r + 1]);
    if (he != hipSuccess) st = hip_fail(he, "hipEventElapsedTime");
    ms.push_back(v);
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st != TS_OK) return st;
  std::sort(ms.begin(), ms.end());
  *seconds = 1e-3 * ms[ms.size() / 2] / inner;
  return TS_OK;
}

// Launches per timed repetition: about a millisecond of work at ~6 TB/s.
int inner_launches(uint64_t bytes) {
  const double est = static_cast<double>(bytes) / 6.0e12 + 5e-6;
  const double r = 1e-3 / est;
  return r < 1 ? 1 : (r > 200 ? 200 : static_cast<int>(r));
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Errors and version
// ---------------------------------------------------------------------------
const char* ts_last_error(void) { return g_error.c_str(); }

int ts_version(int* major, int* minor) {
  if (!major || !minor) return fail(TS_E_INVALID, "NULL out-parameter");
  *major = TS_VERSION_MAJOR;
  *minor = TS_VERSION_MINOR;
  return TS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Targets
// ---------------------------------------------------------------------------
namespace {

int create_target(int device, void* hip_stream, bool owned, ts_target* out) {
  if (!out) return fail(TS_E_INVALID, "NULL out-parameter");
  std::call_once(g_env_cache_once, load_env_cache);
  int count = 0;
  const hipError_t ce = hipGetDeviceCount(&count);
  if (ce != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return fail(TS_E_DEVICE, "no usable GPU: %s", ce != hipSuccess ? hipGetErrorString(ce) : "0 devices");
  }
  if (device < 0 || device >= count)
    return fail(TS_E_INVALID, "device %d out of range (0..%d)", device, count - 1);
  int st = use_device(device);
  if (st != TS_OK) return st;
  hipDeviceProp_t p;
  TS_HIP(hipGetDeviceProperties(&p, device));
  ts_target_s* t = new ts_target_s();
  t->device = device;
  t->info = ts_device_info{};
  t->info.device = device;
  t->info.compute_units = p.multiProcessorCount;
  t->info.wavefront_size = p.warpSize;
  t->info.max_threads_per_block = p.maxThreadsPerBlock;
  t->info.clock_khz = p.clockRate;
  t->info.memory_clock_khz = p.memoryClockRate;
  t->info.memory_bus_width_bits = p.memoryBusWidth;
  t->info.hbm_bytes = p.totalGlobalMem;
  t->info.l2_bytes = static_cast<uint64_t>(p.l2CacheSize);
  t->info.peak_bytes_per_s = kPeakBytesPerS;
  std::snprintf(t->info.arch, sizeof t->info.arch, "%s", p.gcnArchName);
  std::snprintf(t->info.name, sizeof t->info.name, "%s", p.name);
  if (!owned) {
    t->stream = static_cast<hipStream_t>(hip_stream);
    t->owns_stream = false;
  } else {
    const hipError_t e = hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete t;
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
    t->owns_stream = true;
  }
  hipError_t e = hipMalloc(&t->scratch, kReduceScratchBytes);
  if (e == hipSuccess) e = hipHostMalloc(&t->host_result, sizeof(CsPart), hipHostMallocDefault);
  if (e != hipSuccess) {
    if (t->scratch) (void)hipFree(t->scratch);
    if (t->owns_stream) (void)hipStreamDestroy(t->stream);
    delete t;
    return hip_fail(e, "target scratch allocation");
  }
  t->magic = kTargetMagic;
  *out = t;
  return TS_OK;
}

int create_host_target(const int* cpus, int ncpus, ts_target* out) {
  if (!out) return fail(TS_E_INVALID, "NULL out-parameter");
  if (ncpus < 0 || (ncpus > 0 && !cpus)) return fail(TS_E_INVALID, "bad CPU list");
  std::vector<int> list;
  if (ncpus > 0) {
    const std::vector<int> allowed = host_allowed_cpus();
    for (int i = 0; i < ncpus; ++i) {
      if (std::find(allowed.begin(), allowed.end(), cpus[i]) == allowed.end())
        return fail(TS_E_INVALID, "CPU %d is not in the process's affinity set", cpus[i]);
      list.push_back(cpus[i]);
    }
  } else {
    for (const auto& dom : host_domains()) list.insert(list.end(), dom.begin(), dom.end());
  }
  if (list.empty()) return fail(TS_E_INVALID, "no CPU to run on");
  if (list.size() > 4096) return fail(TS_E_INVALID, "too many CPUs");
  ts_target_s* t = new ts_target_s();
  t->device = kHostDevice;
  t->host = true;
  t->pool = new HostPool(list);
  t->stream = nullptr;
  t->owns_stream = false;
  t->info = ts_device_info{};
  t->info.device = kHostDevice;
  t->info.compute_units = static_cast<int>(list.size());
  const long pages = sysconf(_SC_PHYS_PAGES), page = sysconf(_SC_PAGESIZE);
  t->info.hbm_bytes = pages > 0 && page > 0 ? static_cast<uint64_t>(pages) * static_cast<uint64_t>(page) : 0;
  t->info.peak_bytes_per_s = 0.0;  // not known for the host
  std::snprintf(t->info.arch, sizeof t->info.arch, "host");
  std::snprintf(t->info.name, sizeof t->info.name, "host CPUs (%zu pinned workers)", list.size());
  t->magic = kTargetMagic;
  *out = t;
  return TS_OK;
}

}  // namespace

extern "C" {

int ts_target_create_host(const int* cpus, int ncpus, ts_target* out) {
  TS_GUARD_BEGIN
  return create_host_target(cpus, ncpus, out);
  TS_GUARD_END
}

int ts_host_numa_domains(int* count) {
  TS_GUARD_BEGIN
  if (!count) return fail(TS_E_INVALID, "NULL out-parameter");
  *count = static_cast<int>(host_domains().size());
  return TS_OK;
  TS_GUARD_END
}

int ts_host_domain_cpus(int domain, int* cpus, int cap, int* count) {
  TS_GUARD_BEGIN
  if (!count || cap < 0 || (cap > 0 && !cpus)) return fail(TS_E_INVALID, "bad arguments");
  const auto doms = host_domains();
  if (domain < 0 || domain >= static_cast<int>(doms.size())) return fail(TS_E_INVALID, "no such domain");
  const auto& d = doms[static_cast<size_t>(domain)];
  for (int i = 0; i < cap && i < static_cast<int>(d.size()); ++i) cpus[i] = d[static_cast<size_t>(i)];
  *count = static_cast<int>(d.size());
  return TS_OK;
  TS_GUARD_END
}

int ts_target_create(int device, void* hip_stream, ts_target* out) {
  TS_GUARD_BEGIN
  return create_target(device, hip_stream, false, out);
  TS_GUARD_END
}

int ts_target_create_owned(int device, ts_target* out) {
  TS_GUARD_BEGIN
  return create_target(device, nullptr, true, out);
  TS_GUARD_END
}

int ts_target_destroy(ts_target t) {
  if (!t) return TS_OK;
  if (!ok_target(t)) return fail(TS_E_INVALID, "invalid target handle");
  if (t->host) {
    delete t->pool;
    t->magic = kDead;
    delete t;
    return TS_OK;
  }
  (void)use_device(t->device);
  (void)hipStreamSynchronize(t->stream);
  (void)hipFree(t->scratch);
  (void)hipHostFree(t->host_result);
  if (t->owns_stream) (void)hipStreamDestroy(t->stream);
  t->magic = kDead;
  delete t;
  return TS_OK;
}

int ts_target_synchronize(ts_target t) {
  if (!ok_target(t)) return fail(TS_E_INVALID, "invalid target handle");
  if (t->host) return TS_OK;  // host calls complete before they return
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  TS_HIP(hipStreamSynchronize(t->stream));
  return TS_OK;
}

int ts_target_info(ts_target t, ts_device_info* out) {
  if (!ok_target(t) || !out) return fail(TS_E_INVALID, "invalid target handle or NULL out");
  *out = t->info;
  return TS_OK;
}

int ts_target_stream(ts_target t, void** out) {
  if (!ok_target(t) || !out) return fail(TS_E_INVALID, "invalid target handle or NULL out");
  if (t->host) return host_only_gpu("a stream");
  *out = t->stream;
  return TS_OK;
}

int ts_target_then(ts_target t, void (*fn)(void*), void* user) {
  if (!ok_target(t) || !fn) return fail(TS_E_INVALID, "invalid target handle or NULL callback");
  if (t->host) {  // all earlier work has completed: run the continuation now
    fn(user);
    return TS_OK;
  }
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  TS_HIP(hipLaunchHostFunc(t->stream, fn, user));
  return TS_OK;
}

// ---------------------------------------------------------------------------
// Arrays
// ---------------------------------------------------------------------------
int ts_array_alloc(ts_target t, ts_dtype dtype, size_t n, size_t offset_elems, ts_array* out) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !out) return fail(TS_E_INVALID, "invalid target handle or NULL out");
  if (!valid_dtype(dtype)) return fail(TS_E_INVALID, "unknown dtype %d", static_cast<int>(dtype));
  const size_t es = dtype_size(dtype);
  const size_t max_elems = SIZE_MAX / es - 1;
  if (offset_elems > max_elems || n > max_elems - offset_elems) return fail(TS_E_INVALID, "size overflow");
  void* base = nullptr;
  const size_t bytes = (n + offset_elems) * es;
  if (t->host) {
    // Pages are not touched here: bulk construction (ts_fill*) writes each
    // block from its own worker, which places it on that worker's node.
    if (bytes > 0) {
      const size_t rounded = (bytes + 4095) / 4096 * 4096;
      base = std::aligned_alloc(4096, rounded);
      if (!base) return fail(TS_E_OOM, "host allocation of %zu bytes failed", rounded);
    }
  } else if (bytes > 0) {
    int st = use_device(t->device);
    if (st != TS_OK) return st;
    const hipError_t e = hipMalloc(&base, bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    if (reinterpret_cast<uintptr_t>(base) % 256 != 0) {
      (void)hipFree(base);
      return fail(TS_E_DEVICE, "hipMalloc returned a base not aligned to 256 bytes");
    }
  }
  ts_array_s* a = new ts_array_s();
  a->target = t;
  a->device = t->device;
  a->dtype = dtype;
  a->owned_base = base;
  a->ptr = base ? static_cast<char*>(base) + offset_elems * es : nullptr;
  a->n = n;
  a->magic = kArrayMagic;
  *out = a;
  return TS_OK;
  TS_GUARD_END
}

int ts_array_wrap(ts_target t, ts_dtype dtype, void* dev_ptr, size_t n, ts_array* out) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !out) return fail(TS_E_INVALID, "invalid target handle or NULL out");
  if (!valid_dtype(dtype)) return fail(TS_E_INVALID, "unknown dtype %d", static_cast<int>(dtype));
  const size_t es = dtype_size(dtype);
  if (n > 0 && !dev_ptr) return fail(TS_E_INVALID, "NULL pointer with n > 0");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % es != 0)
    return fail(TS_E_INVALID, "pointer not aligned to the element size (%zu bytes)", es);
  if (n > 0 && t->host) {
    // Host targets borrow host memory: refuse memory the HIP runtime knows
    // as device memory (an unknown pointer is ordinary host memory).
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    const hipError_t e = hipPointerGetAttributes(&attr, dev_ptr);
    if (e != hipSuccess) (void)hipGetLastError();
    else if (attr.type == hipMemoryTypeDevice)
      return fail(TS_E_PLACEMENT, "pointer is device memory; a host target needs host memory");
  } else if (n > 0) {
    int st = use_device(t->device);
    if (st != TS_OK) return st;
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    const hipError_t e = hipPointerGetAttributes(&attr, dev_ptr);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(TS_E_PLACEMENT, "pointer is not device memory known to the HIP runtime");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
      return fail(TS_E_PLACEMENT, "pointer is not device memory (memory type %d)", static_cast<int>(attr.type));
    if (attr.device != t->device)
      return fail(TS_E_PLACEMENT, "pointer lives on device %d, the target is device %d", attr.device, t->device);
  }
  ts_array_s* a = new ts_array_s();
  a->target = t;
  a->device = t->device;
  a->dtype = dtype;
  a->ptr = dev_ptr;
  a->n = n;
  a->owned_base = nullptr;
  a->magic = kArrayMagic;
  *out = a;
  return TS_OK;
  TS_GUARD_END
}

int ts_array_free(ts_array a) {
  if (!a) return TS_OK;
  if (!ok_array(a)) return fail(TS_E_INVALID, "invalid array handle");
  if (a->owned_base && a->device == kHostDevice) {
    std::free(a->owned_base);
  } else if (a->owned_base) {
    (void)use_device(a->device);
    (void)hipFree(a->owned_base);
  }
  a->magic = kDead;
  delete a;
  return TS_OK;
}

int ts_array_info(ts_array a, void** ptr, size_t* n, ts_dtype* dtype) {
  if (!ok_array(a)) return fail(TS_E_INVALID, "invalid array handle");
  if (ptr) *ptr = a->ptr;
  if (n) *n = a->n;
  if (dtype) *dtype = static_cast<ts_dtype>(a->dtype);
  return TS_OK;
}

int ts_fill(ts_array a, double value) {
  if (!ok_array(a) || !ok_target(a->target)) return fail(TS_E_INVALID, "invalid array handle");
  if (!map_dtype(a->dtype)) return fail(TS_E_UNSUPPORTED, "fills take floating-point storage");
  if (a->n == 0) return TS_OK;
  if (a->target->host) {
    if (a->dtype == TS_F64)
      host_blocks(a->target, a->n, [&](uint64_t lo, uint64_t hi, int) { host_fill_f64(static_cast<double*>(a->ptr), lo, hi, value); });
    else if (a->dtype == TS_F32)
      host_blocks(a->target, a->n, [&](uint64_t lo, uint64_t hi, int) {
        host_fill_f32(static_cast<float*>(a->ptr), lo, hi, static_cast<float>(value));
      });
    else
      return fail(TS_E_UNSUPPORTED, "host targets support binary64 and binary32 storage");
    return TS_OK;
  }
  int st = use_device(a->device);
  if (st != TS_OK) return st;
  const hipError_t e = launch_fill_const(a->dtype, a->ptr, a->n, value, a->target->stream);
  if (e != hipSuccess) return hip_fail(e, "fill kernel launch");
  return TS_OK;
}

int ts_fill_uniform_range(ts_array a, uint64_t seed, uint64_t stream_id, uint64_t first_index, double vlo,
                          double vhi) {
  if (!ok_array(a) || !ok_target(a->target)) return fail(TS_E_INVALID, "invalid array handle");
  if (!map_dtype(a->dtype)) return fail(TS_E_UNSUPPORTED, "fills take floating-point storage");
  if (stream_id >= (1ull << 16)) return fail(TS_E_INVALID, "stream_id must be below 2^16");
  const double w = vhi - vlo;
  if (!(vlo < vhi) || !std::isfinite(vlo) || !std::isfinite(vhi) || !std::isfinite(w))
    return fail(TS_E_INVALID, "the range needs finite lo < hi with a finite difference");
  if (a->n == 0) return TS_OK;
  if (a->target->host) {
    const uint64_t state0 = seed ^ (stream_id << 48);
    if (a->dtype == TS_F64)
      host_blocks(a->target, a->n, [&](uint64_t lo, uint64_t hi, int) {
        host_fill_uniform_f64(static_cast<double*>(a->ptr), lo, hi, state0, first_index, vlo, w);
      });
    else if (a->dtype == TS_F32)
      host_blocks(a->target, a->n, [&](uint64_t lo, uint64_t hi, int) {
        host_fill_uniform_f32(static_cast<float*>(a->ptr), lo, hi, state0, first_index, vlo, w);
      });
    else
      return fail(TS_E_UNSUPPORTED, "host targets support binary64 and binary32 storage");
    return TS_OK;
  }
  int st = use_device(a->device);
  if (st != TS_OK) return st;
  const hipError_t e =
      launch_fill_uniform(a->dtype, a->ptr, a->n, seed, stream_id, first_index, vlo, w, a->target->stream);
  if (e != hipSuccess) return hip_fail(e, "uniform fill kernel launch");
  return TS_OK;
}

int ts_fill_uniform(ts_array a, uint64_t seed, uint64_t stream_id, uint64_t first_index) {
  return ts_fill_uniform_range(a, seed, stream_id, first_index, -1.0, 1.0);
}

int ts_copy_from_host(ts_array dst, const void* src, size_t n) {
  if (!ok_array(dst) || !ok_target(dst->target)) return fail(TS_E_INVALID, "invalid array handle");
  if (n > dst->n) return fail(TS_E_SHAPE, "%zu elements do not fit an array of %llu", n,
                              static_cast<unsigned long long>(dst->n));
  if (n == 0) return TS_OK;
  if (!src) return fail(TS_E_INVALID, "NULL host pointer");
  if (dst->target->host) {
    std::memcpy(dst->ptr, src, n * dtype_size(dst->dtype));
    return TS_OK;
  }
  int st = use_device(dst->device);
  if (st != TS_OK) return st;
  TS_HIP(hipMemcpyAsync(dst->ptr, src, n * dtype_size(dst->dtype), hipMemcpyHostToDevice,
                        dst->target->stream));
  return TS_OK;
}

int ts_copy_to_host(void* dst, ts_array src, size_t n) {
  if (!ok_array(src) || !ok_target(src->target)) return fail(TS_E_INVALID, "invalid array handle");
  if (n > src->n) return fail(TS_E_SHAPE, "%zu elements exceed an array of %llu", n,
                              static_cast<unsigned long long>(src->n));
  if (n == 0) return TS_OK;
  if (!dst) return fail(TS_E_INVALID, "NULL host pointer");
  if (src->target->host) {
    std::memcpy(dst, src->ptr, n * dtype_size(src->dtype));
    return TS_OK;
  }
  int st = use_device(src->device);
  if (st != TS_OK) return st;
  TS_HIP(hipMemcpyAsync(dst, src->ptr, n * dtype_size(src->dtype), hipMemcpyDeviceToHost,
                        src->target->stream));
  return TS_OK;
}

// ---------------------------------------------------------------------------
// Algorithms
// ---------------------------------------------------------------------------
int ts_copy(ts_target exec, ts_array src, ts_array dst) {
  TS_GUARD_BEGIN
  return run_map(exec, TS_COPY, src, nullptr, dst, 0.0);
  TS_GUARD_END
}

int ts_scale(ts_target exec, ts_array src, ts_array dst, double q) {
  TS_GUARD_BEGIN
  return run_map(exec, TS_SCALE, src, nullptr, dst, q);
  TS_GUARD_END
}

int ts_add(ts_target exec, ts_array x, ts_array y, ts_array dst) {
  TS_GUARD_BEGIN
  return run_map(exec, TS_ADD, x, y, dst, 0.0);
  TS_GUARD_END
}

int ts_triad(ts_target exec, ts_array x, ts_array y, ts_array dst, double q) {
  TS_GUARD_BEGIN
  return run_map(exec, TS_TRIAD, x, y, dst, q);
  TS_GUARD_END
}

int ts_stream_iteration(ts_target exec, ts_array a, ts_array b, ts_array c, double q) {
  TS_GUARD_BEGIN
  if (!ok_target(exec)) return fail(TS_E_INVALID, "invalid target handle");
  if (!ok_array(a) || !ok_array(b) || !ok_array(c)) return fail(TS_E_INVALID, "invalid array handle");
  const size_t es = dtype_size(a->dtype);
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a->ptr), pb = reinterpret_cast<uintptr_t>(b->ptr),
                  pc = reinterpret_cast<uintptr_t>(c->ptr);
  if (ranges_overlap(pa, pb, a->n, es) || ranges_overlap(pa, pc, a->n, es) ||
      ranges_overlap(pb, pc, a->n, es))
    return fail(TS_E_ALIAS, "the benchmark arrays a, b, c must not overlap");
  // All four maps are checked before any is enqueued, so an error leaves the
  // arrays untouched.
  uint64_t count = 0;
  int st;
  if ((st = check_exec_arrays(exec, TS_COPY, a, nullptr, c, &count)) != TS_OK ||
      (st = check_exec_arrays(exec, TS_SCALE, c, nullptr, b, &count)) != TS_OK ||
      (st = check_exec_arrays(exec, TS_ADD, a, b, c, &count)) != TS_OK ||
      (st = check_exec_arrays(exec, TS_TRIAD, b, c, a, &count)) != TS_OK)
    return st;
  if (!map_dtype(a->dtype)) return fail(TS_E_UNSUPPORTED, "the STREAM maps take floating-point storage");
  if ((st = run_map(exec, TS_COPY, a, nullptr, c, q)) != TS_OK) return st;   // c = a
  if ((st = run_map(exec, TS_SCALE, c, nullptr, b, q)) != TS_OK) return st;  // b = q*c
  if ((st = run_map(exec, TS_ADD, a, b, c, q)) != TS_OK) return st;          // c = a + b
  return run_map(exec, TS_TRIAD, b, c, a, q);                                // a = b + q*c
  TS_GUARD_END
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
int ts_checksum(ts_target t, ts_array x, double expected, ts_checksum_out* out) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !ok_array(x) || !out) return fail(TS_E_INVALID, "invalid handle or NULL out");
  if (!map_dtype(x->dtype)) return fail(TS_E_UNSUPPORTED, "checksums take floating-point storage");
  if (x->device != t->device) return fail(TS_E_PLACEMENT, "array is not on the executor's device");
  if (x->n == 0) {
    *out = ts_checksum_out{0.0, 0.0, 0.0, 0};
    return TS_OK;
  }
  if (t->host) {
    if (x->dtype != TS_F64 && x->dtype != TS_F32)
      return fail(TS_E_UNSUPPORTED, "host targets support binary64 and binary32 storage");
    std::vector<HostPart> parts(static_cast<size_t>(t->pool->size()));
    host_blocks(t, x->n, [&](uint64_t lo, uint64_t hi, int w) {
      parts[static_cast<size_t>(w)] = x->dtype == TS_F64
          ? host_checksum_f64(static_cast<const double*>(x->ptr), lo, hi, expected)
          : host_checksum_f32(static_cast<const float*>(x->ptr), lo, hi, expected);
    });
    ts_checksum_out r{0.0, 0.0, std::nan(""), 0};
    for (const HostPart& p : parts) {  // fixed order: worker 0, 1, ...
      r.sum += p.sum;
      r.abs_dev_sum += p.absdev;
      r.max_abs_dev = std::fmax(r.max_abs_dev, p.maxdev);
      r.mismatches += p.mism;
    }
    *out = r;
    return TS_OK;
  }
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  hipError_t e = launch_checksum(x->dtype, x->ptr, x->n, expected, t->scratch, t->stream);
  if (e != hipSuccess) return hip_fail(e, "checksum kernel launch");
  const CsPart* res = static_cast<const CsPart*>(t->scratch) + kReduceMaxParts;
  TS_HIP(hipMemcpyAsync(t->host_result, res, sizeof(CsPart), hipMemcpyDeviceToHost, t->stream));
  TS_HIP(hipStreamSynchronize(t->stream));
  const CsPart* h = static_cast<const CsPart*>(t->host_result);
  *out = ts_checksum_out{h->sum, h->absdev, h->maxdev, h->mism};
  return TS_OK;
  TS_GUARD_END
}

int ts_mismatch_count(ts_target t, ts_array x, ts_array ref, uint64_t* out) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !ok_array(x) || !ok_array(ref) || !out)
    return fail(TS_E_INVALID, "invalid handle or NULL out");
  if (x->dtype != ref->dtype) return fail(TS_E_DTYPE, "arrays of different storage types");
  if (!map_dtype(x->dtype)) return fail(TS_E_UNSUPPORTED, "mismatch counts take floating-point storage");
  if (x->device != t->device || ref->device != t->device)
    return fail(TS_E_PLACEMENT, "array is not on the executor's device");
  if (ref->n < x->n) return fail(TS_E_SHAPE, "ref holds fewer elements than x");
  if (x->n == 0) {
    *out = 0;
    return TS_OK;
  }
  if (t->host) {
    if (x->dtype != TS_F64 && x->dtype != TS_F32)
      return fail(TS_E_UNSUPPORTED, "host targets support binary64 and binary32 storage");
    std::vector<uint64_t> parts(static_cast<size_t>(t->pool->size()), 0);
    const size_t es = dtype_size(x->dtype);
    host_blocks(t, x->n, [&](uint64_t lo, uint64_t hi, int w) {
      parts[static_cast<size_t>(w)] = host_mismatch(x->ptr, ref->ptr, lo, hi, es, x->dtype == TS_F64);
    });
    uint64_t total = 0;
    for (uint64_t c : parts) total += c;
    *out = total;
    return TS_OK;
  }
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  hipError_t e = launch_mismatch(x->dtype, x->ptr, ref->ptr, x->n, t->scratch, t->stream);
  if (e != hipSuccess) return hip_fail(e, "mismatch kernel launch");
  const CsPart* res = static_cast<const CsPart*>(t->scratch) + kReduceMaxParts;
  TS_HIP(hipMemcpyAsync(t->host_result, res, sizeof(CsPart), hipMemcpyDeviceToHost, t->stream));
  TS_HIP(hipStreamSynchronize(t->stream));
  *out = static_cast<const CsPart*>(t->host_result)->mism;
  return TS_OK;
  TS_GUARD_END
}

// ---------------------------------------------------------------------------
// Launch configuration and tuning
// ---------------------------------------------------------------------------
int ts_get_kernel_cfg(ts_op op, ts_dtype dtype, size_t n, int align_class, int batched,
                      ts_kernel_cfg* out) {
  TS_GUARD_BEGIN
  if (!valid_op(op) || !map_dtype(dtype) || !out || align_class < 0 || align_class > 2)
    return fail(TS_E_INVALID, "bad op, dtype, alignment class or NULL out");
  ts_kernel_cfg c = tune_table().lookup(op, dtype, n, align_class, batched ? 1 : 0);
  if (!batched && c.vec_bytes == 0) c.vec_bytes = static_cast<int32_t>(dtype_size(dtype));
  *out = c;
  return TS_OK;
  TS_GUARD_END
}

int ts_set_kernel_cfg(ts_op op, ts_dtype dtype, int batched, const ts_kernel_cfg* cfg) {
  TS_GUARD_BEGIN
  if (!valid_op(op) || !map_dtype(dtype)) return fail(TS_E_INVALID, "bad op or dtype");
  if (cfg) {
    const std::string why = cfg_problem(*cfg, batched ? 1 : 0);
    if (!why.empty()) return fail(TS_E_INVALID, "invalid configuration: %s", why.c_str());
  }
  tune_table().force(op, dtype, batched ? 1 : 0, cfg);
  return TS_OK;
  TS_GUARD_END
}

int ts_autotune_candidates(int batched, ts_kernel_cfg* out, size_t cap, size_t* count) {
  TS_GUARD_BEGIN
  if (!count) return fail(TS_E_INVALID, "NULL count");
  const std::vector<ts_kernel_cfg> c = candidates(batched ? 1 : 0);
  if (out)
    for (size_t i = 0; i < c.size() && i < cap; ++i) out[i] = c[i];
  *count = c.size();
  return TS_OK;
  TS_GUARD_END
}

int ts_autotune(ts_target t, ts_op op, ts_dtype dtype, size_t n, size_t offset_elems, int reps,
                ts_kernel_cfg* best, double* best_bytes_per_s) {
  TS_GUARD_BEGIN
  if (!ok_target(t)) return fail(TS_E_INVALID, "invalid target handle");
  if (t->host) return host_only_gpu("tuning");
  if (!valid_op(op) || !map_dtype(dtype) || n == 0)
    return fail(TS_E_INVALID, "bad op, dtype or zero size");
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  const size_t es = dtype_size(dtype);
  void* base[3] = {nullptr, nullptr, nullptr};
  for (int i = 0; i < 3; ++i) {
    const hipError_t e = hipMalloc(&base[i], (n + offset_elems) * es);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipFree(base[j]);
      return hip_fail(e, "hipMalloc (autotune arrays)");
    }
  }
  char* p[3];
  for (int i = 0; i < 3; ++i) {
    p[i] = static_cast<char*>(base[i]) + offset_elems * es;
    if (st == TS_OK) {
      const hipError_t e =
          launch_fill_uniform(dtype, p[i], n, 1, static_cast<uint64_t>(i), 0, -1.0, 2.0, t->stream);
      if (e != hipSuccess) st = hip_fail(e, "fill kernel launch");
    }
  }
  const bool has_y = op == TS_ADD || op == TS_TRIAD;
  const uintptr_t ya = reinterpret_cast<uintptr_t>(p[1]);
  const int cls = align_class(reinterpret_cast<uintptr_t>(p[0]), has_y ? &ya : nullptr,
                              reinterpret_cast<uintptr_t>(p[2]));
  ts_kernel_cfg best_cfg = default_cfg(0, dtype);
  double best_s = 0;
  const uint64_t bytes = stream_bytes(op, n, es);
  for (const ts_kernel_cfg& c : candidates(0)) {
    if (st != TS_OK) break;
    double s = 0;
    st = time_candidate(t, reps, inner_launches(bytes),
                        [&]() { return launch_map(t, op, dtype, p[0], p[1], p[2], n, 3.0, c); }, &s);
    if (st == TS_OK && s > 0 && (best_s == 0 || s < best_s)) {
      best_s = s;
      best_cfg = c;
    }
  }
  (void)hipStreamSynchronize(t->stream);
  for (int i = 0; i < 3; ++i) (void)hipFree(base[i]);
  if (st != TS_OK) return st;
  const double bps = best_s > 0 ? static_cast<double>(bytes) / best_s : 0.0;
  tune_table().put(TuneKey{op, dtype, size_bucket(n), cls, 0}, TuneEntry{best_cfg, bps});
  if (best) *best = best_cfg;
  if (best_bytes_per_s) *best_bytes_per_s = bps;
  return TS_OK;
  TS_GUARD_END
}

int ts_autotune_batch(ts_target t, ts_batch b, ts_op op, int reps, ts_kernel_cfg* best,
                      double* best_bytes_per_s) {
  TS_GUARD_BEGIN
  int st = check_batch_exec(t, b);
  if (st != TS_OK) return st;
  if (!valid_op(op)) return fail(TS_E_INVALID, "bad op");
  if (b->total == 0) return fail(TS_E_INVALID, "empty batch");
  const int64_t original_tile = b->tile_elems;
  const bool pinned = b->tile_pinned;
  free_op_plans(b);
  b->tile_pinned = true;  // candidates run on the primary plan, re-planned to their tile
  ts_kernel_cfg best_cfg = default_cfg(1, b->dtype);
  double best_s = 0;
  for (const ts_kernel_cfg& c : candidates(1)) {
    if (c.tile_elems != b->tile_elems && (st = batch_replan(b, c.tile_elems)) != TS_OK) break;
    double s = 0;
    st = time_candidate(t, reps, 1, [&]() { return launch_batch(t, b, op, c); }, &s);
    if (st != TS_OK) break;
    if (s > 0 && (best_s == 0 || s < best_s)) {
      best_s = s;
      best_cfg = c;
    }
  }
  const double bps =
      best_s > 0 ? static_cast<double>(stream_bytes(op, b->total, dtype_size(b->dtype))) / best_s : 0.0;
  if (st == TS_OK)
    tune_table().put(TuneKey{op, b->dtype, size_bucket(b->total), TS_ALIGN_16, 1}, TuneEntry{best_cfg, bps});
  // Back to the batch's own tile; the maps' plans now follow the updated table.
  b->tile_pinned = pinned;
  const int rst = batch_replan(b, original_tile);
  if (st != TS_OK) return st;
  if (rst != TS_OK) return rst;
  if ((st = build_op_plans(b)) != TS_OK) return st;
  if (best) *best = best_cfg;
  if (best_bytes_per_s) *best_bytes_per_s = bps;
  return TS_OK;
  TS_GUARD_END
}

int ts_tune_cache_load(const char* path) {
  TS_GUARD_BEGIN
  if (!path) return fail(TS_E_INVALID, "NULL path");
  std::string err;
  if (tune_table().load(path, &err) != 0) return fail(TS_E_INVALID, "%s", err.c_str());
  return TS_OK;
  TS_GUARD_END
}

int ts_tune_cache_save(const char* path) {
  TS_GUARD_BEGIN
  if (!path) return fail(TS_E_INVALID, "NULL path");
  std::string err;
  if (tune_table().save(path, &err) != 0) return fail(TS_E_INVALID, "%s", err.c_str());
  return TS_OK;
  TS_GUARD_END
}

int ts_tune_cache_clear(void) {
  TS_GUARD_BEGIN
  tune_table().clear();
  return TS_OK;
  TS_GUARD_END
}

int ts_time_op(ts_target exec, ts_op op, ts_array x, ts_array y, ts_array dst, double q, int reps,
               float* ms_total) {
  TS_GUARD_BEGIN
  if (!valid_op(op) || !ms_total || reps < 1) return fail(TS_E_INVALID, "bad op, reps or NULL out");
  uint64_t count = 0;
  int st = check_exec_arrays(exec, op, x, y, dst, &count);
  if (st != TS_OK) return st;
  if (exec->host) {
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps && st == TS_OK; ++r) st = run_map(exec, op, x, y, dst, q);
    if (st != TS_OK) return st;
    *ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return TS_OK;
  }
  if ((st = use_device(exec->device)) != TS_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TS_HIP(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he, "hipEventCreate");
  }
  he = hipEventRecord(e0, exec->stream);
  for (int r = 0; r < reps && he == hipSuccess && st == TS_OK; ++r) st = run_map(exec, op, x, y, dst, q);
  if (he == hipSuccess && st == TS_OK) he = hipEventRecord(e1, exec->stream);
  if (he == hipSuccess && st == TS_OK) he = hipEventSynchronize(e1);
  float ms = 0;
  if (he == hipSuccess && st == TS_OK) he = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TS_OK) return st;
  if (he != hipSuccess) return hip_fail(he, "event timing");
  *ms_total = ms;
  return TS_OK;
  TS_GUARD_END
}

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
  const size_t es = dtype_size(dtype);
  // Placement: every instance's first element must be device memory of this
  // device (one query per array; instances are not required to be distinct
  // allocations).
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
    delete b;
    return status;
  };
  std::vector<uintptr_t> seen;
  for (size_t i = 0; i < count; ++i) {
    if (descs[i].len == 0) continue;
    for (void* ptr : {descs[i].a, descs[i].b, descs[i].c}) {
      if (!ptr) return cleanup(fail(TS_E_INVALID, "instance %zu: NULL array with len > 0", i));
      hipPointerAttribute_t attr;
      std::memset(&attr, 0, sizeof attr);
      const hipError_t e = hipPointerGetAttributes(&attr, ptr);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(TS_E_PLACEMENT, "instance %zu: pointer is not device memory", i));
      }
      if ((attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) ||
          attr.device != t->device)
        return cleanup(fail(TS_E_PLACEMENT, "instance %zu: array is not on the target's device", i));
    }
  }
  (void)es;
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
  const hipError_t e = launch_batch_fill(b->dtype, b->d_tiles, b->tiles.size(), which, 0,
                                         value, 0, aux_grid(exec, b->tiles.size()), exec->stream);
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
  const hipError_t e = launch_batch_fill(b->dtype, b->d_tiles, b->tiles.size(), which, 1,
                                         0.0, seed, aux_grid(exec, b->tiles.size()), exec->stream);
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
  TS_HIP(hipMemcpyAsync(b->d_expected, expected, n * sizeof(double), hipMemcpyHostToDevice, exec->stream));
  hipError_t e = launch_zero_u64(b->d_counts, n, exec->stream);
  if (e != hipSuccess) return hip_fail(e, "zero kernel launch");
  if (!b->tiles.empty()) {
    e = launch_batch_mismatch(b->dtype, b->d_tiles, b->tiles.size(), which, b->d_expected,
                              b->d_counts, aux_grid(exec, b->tiles.size()), exec->stream);
    if (e != hipSuccess) return hip_fail(e, "batched mismatch launch");
  }
  TS_HIP(hipMemcpyAsync(counts, b->d_counts, n * sizeof(uint64_t), hipMemcpyDeviceToHost, exec->stream));
  TS_HIP(hipStreamSynchronize(exec->stream));
  return TS_OK;
  TS_GUARD_END
}

// ---------------------------------------------------------------------------
// Graphs
// ---------------------------------------------------------------------------
}  // extern "C"

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
  return capture(
      t,
      [&]() {
        for (int k = 0; k < iterations; ++k) {
          const int s = ts_stream_iteration(t, a, b, c, q);
          if (s != TS_OK) return s;
        }
        return static_cast<int>(TS_OK);
      },
      out);
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
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  g->magic = kDead;
  delete g;
  return TS_OK;
}

// ---------------------------------------------------------------------------
// Events
// ---------------------------------------------------------------------------
int ts_event_create(ts_event* out) {
  TS_GUARD_BEGIN
  if (!out) return fail(TS_E_INVALID, "NULL out");
  int dev = 0;
  TS_HIP(hipGetDevice(&dev));
  hipEvent_t ev = nullptr;
  TS_HIP(hipEventCreate(&ev));
  ts_event_s* e = new ts_event_s();
  e->device = dev;
  e->ev = ev;
  e->recorded = false;
  e->magic = kEventMagic;
  *out = e;
  return TS_OK;
  TS_GUARD_END
}

int ts_event_destroy(ts_event e) {
  if (!e) return TS_OK;
  if (!ok_event(e)) return fail(TS_E_INVALID, "invalid event handle");
  (void)hipEventDestroy(e->ev);
  e->magic = kDead;
  delete e;
  return TS_OK;
}

int ts_event_record(ts_event e, ts_target t) {
  if (!ok_event(e) || !ok_target(t)) return fail(TS_E_INVALID, "invalid event or target handle");
  if (t->host) return host_only_gpu("events");
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  TS_HIP(hipEventRecord(e->ev, t->stream));
  e->recorded = true;
  return TS_OK;
}

int ts_event_synchronize(ts_event e) {
  if (!ok_event(e)) return fail(TS_E_INVALID, "invalid event handle");
  TS_HIP(hipEventSynchronize(e->ev));
  return TS_OK;
}

int ts_event_query(ts_event e) {
  if (!ok_event(e)) return fail(TS_E_INVALID, "invalid event handle");
  const hipError_t r = hipEventQuery(e->ev);
  if (r == hipSuccess) return TS_OK;
  if (r == hipErrorNotReady) {
    (void)hipGetLastError();
    return 1;
  }
  return hip_fail(r, "hipEventQuery");
}

int ts_event_elapsed_ms(ts_event start, ts_event end, float* ms) {
  if (!ok_event(start) || !ok_event(end) || !ms) return fail(TS_E_INVALID, "invalid event handle or NULL out");
  TS_HIP(hipEventElapsedTime(ms, start->ev, end->ev));
  return TS_OK;
}

// ---------------------------------------------------------------------------
// Futures
// ---------------------------------------------------------------------------
int ts_target_async(ts_target t, ts_future* out) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !out) return fail(TS_E_INVALID, "invalid target handle or NULL out");
  ts_future_s* f = new ts_future_s();
  f->ready = false;
  f->magic = kFutureMagic;
  if (t->host) {  // host calls complete before they return
    f->ready = true;
    *out = f;
    return TS_OK;
  }
  int st = use_device(t->device);
  if (st != TS_OK) {
    f->magic = kDead;
    delete f;
    return st;
  }
  const hipError_t e = hipLaunchHostFunc(t->stream, future_ready_cb, f);
  if (e != hipSuccess) {
    f->magic = kDead;
    delete f;
    return hip_fail(e, "hipLaunchHostFunc");
  }
  *out = f;
  return TS_OK;
  TS_GUARD_END
}

int ts_future_wait(ts_future f) {
  TS_GUARD_BEGIN
  if (!ok_future(f)) return fail(TS_E_INVALID, "invalid future handle");
  std::unique_lock<std::mutex> lk(f->mu);
  f->cv.wait(lk, [f] { return f->ready; });
  return TS_OK;
  TS_GUARD_END
}

int ts_future_ready(ts_future f) {
  TS_GUARD_BEGIN
  if (!ok_future(f)) return fail(TS_E_INVALID, "invalid future handle");
  std::lock_guard<std::mutex> lk(f->mu);
  return f->ready ? 1 : 0;
  TS_GUARD_END
}

int ts_future_destroy(ts_future f) {
  if (!f) return TS_OK;
  if (!ok_future(f)) return fail(TS_E_INVALID, "invalid future handle");
  {
    std::unique_lock<std::mutex> lk(f->mu);
    f->cv.wait(lk, [f] { return f->ready; });  // the callback still refers to it
  }
  f->magic = kDead;
  delete f;
  return TS_OK;
}

}  // extern "C"
