// capi_tune.cpp -- launch configuration and tuning entry points of the C
// ABI: the configuration table (tuned, forced or default), the autotuner for
// plain and batched maps, its JSON cache, and event-timed runs of a map.
#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "capi_internal.hpp"

using namespace ts;
using namespace tsapi;

namespace {

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
    const hipError_t he = hipEventCreateWithFlags(&e, kTimingEventFlags);
    if (he != hipSuccess) {
      st = hip_fail(he, "hipEventCreateWithFlags");
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
  // Candidates grouped by tile size (one re-plan per size); shapes whose last
  // unrolled vector lies past every full tile are skipped for this storage
  // type (they repeat the shape with a smaller unroll).
  std::vector<ts_kernel_cfg> cands = candidates(1);
  std::stable_sort(cands.begin(), cands.end(),
                   [](const ts_kernel_cfg& x, const ts_kernel_cfg& y) { return x.tile_elems < y.tile_elems; });
  const int64_t per_vec = static_cast<int64_t>(16 / dtype_size(b->dtype));
  for (const ts_kernel_cfg& c : cands) {
    if (static_cast<int64_t>(c.unroll - 1) * c.block * per_vec >= c.tile_elems) continue;
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
  TS_HIP(hipEventCreateWithFlags(&e0, kTimingEventFlags));
  hipError_t he = hipEventCreateWithFlags(&e1, kTimingEventFlags);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he, "hipEventCreateWithFlags");
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

}  // extern "C"
