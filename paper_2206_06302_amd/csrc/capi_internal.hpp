// capi_internal.hpp -- internals shared by the translation units that
// implement the C ABI of libtstream (capi.cpp: errors, targets, arrays,
// algorithms, validation; capi_tune.cpp: launch configuration and tuning;
// capi_batch.cpp: batches and graphs; capi_async.cpp: events and futures).
// Not part of the public interface; every symbol here has hidden visibility.
#pragma once

#include <hip/hip_runtime_api.h>

#include <stddef.h>
#include <stdint.h>

#include <condition_variable>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tstream.h"
#include "host_target.hpp"
#include "ts_handles.hpp"
#include "ts_internal.hpp"
#include "ts_layout.hpp"
#include "tune.hpp"

namespace tsapi {

// Events that only time work: no system-scope release when recorded.
constexpr unsigned kTimingEventFlags = hipEventDisableSystemFence;
constexpr uint32_t kBatchMagic = 0x42415431u;
constexpr uint32_t kGraphMagic = 0x47524631u;
constexpr uint32_t kEventMagic = 0x45564e31u;
constexpr uint32_t kFutureMagic = 0x46555431u;
constexpr uint32_t kDead = 0xdeadbeefu;
constexpr uint64_t kDeadEpoch = ~0ull;
constexpr double kPeakBytesPerS = 8.0e12;  // MI355X HBM3E, the % of peak denominator
constexpr int kHostDevice = -1;

// Record `fmt` for ts_last_error() and return `status`.
int fail(int status, const char* fmt, ...);
// Map a HIP error to TS_E_OOM / TS_E_DEVICE with its text.
int hip_fail(hipError_t e, const char* what);

}  // namespace tsapi

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

struct ts_batch_s {
  uint32_t magic;
  ts_target_s* target;
  int device;
  int dtype;
  std::vector<ts::HostDesc> host;
  std::vector<ts::BatchDesc> descs;  // host-side metadata (alignment per instance)
  std::vector<ts::BatchTile> tiles;  // primary plan: fills, mismatch counts, info
  ts::BatchTile* d_tiles;
  double* d_expected;
  unsigned long long* d_counts;
  // Pinned host staging for the mismatch count's expected values and
  // counts: copies from pageable memory are staged by the runtime on every
  // call, which cost more than the count itself.
  double* h_expected;
  unsigned long long* h_counts;
  uint64_t total;
  int64_t tile_elems;
  // Device plans for the other tile sizes that the maps' tuned configurations
  // ask for, so that each map runs on its own tiles.
  struct OpPlan {
    int64_t tile_elems;
    uint64_t ntiles;
    ts::BatchTile* d_tiles;
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
  std::vector<std::shared_ptr<bool>> arrays_alive;  // graphs of plain arrays
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

namespace tsapi {

inline bool ok_target(const ts_target_s* t) { return t && t->magic == ts::kTargetMagic; }
inline bool ok_array(const ts_array_s* a) { return a && a->magic == ts::kArrayMagic; }
inline bool ok_batch(const ts_batch_s* b) { return b && b->magic == kBatchMagic; }
inline bool ok_graph(const ts_graph_s* g) { return g && g->magic == kGraphMagic; }
inline bool ok_event(const ts_event_s* e) { return e && e->magic == kEventMagic; }
inline bool ok_future(const ts_future_s* f) { return f && f->magic == kFutureMagic; }

int host_only_gpu(const char* what);

// Run fn(lo, hi, w) on every worker of a host target over its block of n.
template <class F>
void host_blocks(ts_target_s* t, uint64_t n, F&& fn) {
  const int W = t->pool->size();
  t->pool->run([&](int w) {
    uint64_t lo, hi;
    ts::HostPool::block(n, W, w, &lo, &hi);
    fn(lo, hi, w);
  });
}

// Stream callback that makes a future ready (runs on a runtime thread).
void future_ready_cb(void* p);
// Make `device` current for the calling thread (cheap when it already is).
int use_device(int device);
// `ptr` must be device memory of `device` whose allocation holds n elements
// of es bytes from ptr on: TS_E_PLACEMENT (not device memory, another device,
// unknown allocation) or TS_E_SHAPE (the allocation ends before n elements).
int check_device_range(int device, const void* ptr, uint64_t n, size_t es, const char* what);
// Storage types of arrays (bytes included) and of the STREAM maps.
bool valid_dtype(int dt);
bool map_dtype(int dt);
bool valid_op(int op);
uint64_t stream_bytes(int op, uint64_t n, size_t es);
hipError_t plain_launch(int dtype, const ts::PlainLaunch& L);
hipError_t batch_launch(int dtype, const ts::BatchLaunch& L);
ts::Operand operand_of(const ts_array_s* a);
// Launch one map over `count` elements with configuration `cfg`.
int launch_map(ts_target_s* t, int op, int dtype, const void* x, const void* y, void* d, uint64_t count,
               double q, const ts_kernel_cfg& cfg);
int check_exec_arrays(ts_target_s* t, int op, ts_array_s* x, ts_array_s* y, ts_array_s* d, uint64_t* count);
int run_map(ts_target_s* t, int op, ts_array_s* x, ts_array_s* y, ts_array_s* d, double q);
// With TS_LOG set (non-empty, not "0"), report on stderr, once per key
// (map, type, size bucket, alignment class, batched), the launch
// configuration the library picked.
void log_choice(int op, int dtype, uint64_t n, int align, int batched, const ts_kernel_cfg& c);

// Batches (capi_batch.cpp).
void bump_epoch(ts_batch_s* b);
int upload_tiles(ts_target_s* t, const std::vector<ts::BatchTile>& tiles, ts::BatchTile** out);
int batch_replan(ts_batch_s* b, int64_t tile_elems);
void free_op_plans(ts_batch_s* b);
ts_kernel_cfg batch_cfg(const ts_batch_s* b, int op);
int build_op_plans(ts_batch_s* b);
int launch_batch(ts_target_s* t, ts_batch_s* b, int op, const ts_kernel_cfg& cfg);
int check_batch_exec(ts_target_s* t, ts_batch_s* b);
// Tiles per workgroup of a batch's fills and mismatch counts, and their grid.
uint32_t aux_tiles_per_wg(const ts_batch_s* b);
uint32_t aux_grid(uint64_t ntiles, uint32_t per_wg);

}  // namespace tsapi
