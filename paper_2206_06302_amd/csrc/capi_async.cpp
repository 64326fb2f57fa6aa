// capi_async.cpp -- completion of enqueued work in the C ABI: events on a
// target's stream, and futures made ready by a stream callback (the
// asynchronous executor functions of Listing 2; the GPU executor signals
// completion with a stream callback, Section 4.2).
#include <chrono>
#include <condition_variable>
#include <mutex>

#include "capi_internal.hpp"

using namespace ts;
using namespace tsapi;

namespace tsapi {

// Notifies while holding the lock: ts_future_destroy may free the future as
// soon as it sees `ready`, so the callback must not touch it after unlocking.
void future_ready_cb(void* p) {
  ts_future_s* f = static_cast<ts_future_s*>(p);
  std::lock_guard<std::mutex> lk(f->mu);
  f->ready = true;
  f->cv.notify_all();
}

}  // namespace tsapi

extern "C" {

// ---------------------------------------------------------------------------
// Events
// ---------------------------------------------------------------------------
namespace {
int event_create(ts_event* out, unsigned flags) {
  TS_GUARD_BEGIN
  if (!out) return fail(TS_E_INVALID, "NULL out");
  int dev = 0;
  TS_HIP(hipGetDevice(&dev));
  hipEvent_t ev = nullptr;
  TS_HIP(hipEventCreateWithFlags(&ev, flags));
  ts_event_s* e = new ts_event_s();
  e->device = dev;
  e->ev = ev;
  e->recorded = false;
  e->magic = kEventMagic;
  *out = e;
  return TS_OK;
  TS_GUARD_END
}
}  // namespace

int ts_event_create(ts_event* out) { return event_create(out, hipEventDefault); }

int ts_event_create_timing(ts_event* out) { return event_create(out, kTimingEventFlags); }

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
