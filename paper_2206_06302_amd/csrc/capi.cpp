// capi.cpp -- the C ABI of libtstream (declared in include/tstream.h):
// errors, targets, arrays, algorithms and validation.
//
// Targets pair a device with a stream (Sections 3.1 and 4.2); arrays are
// placed on a target's device and bulk-constructed there (Section 3.2);
// each algorithm call is one bulk launch on the executing target's stream
// (Sections 3.3 and 3.4).  Every entry point catches everything, returns a
// status and leaves a thread-local message on failure.
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <set>
#include <tuple>

#include "capi_internal.hpp"

using namespace ts;

namespace tsapi {

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

int host_only_gpu(const char* what) {
  return fail(TS_E_UNSUPPORTED, "%s needs a GPU target (this is a host-CPU target)", what);
}

// Make `device` current for the calling thread (cheap when it already is).
int check_device_range(int device, const void* ptr, uint64_t n, size_t es, const char* what) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TS_E_PLACEMENT, "%s: pointer is not device memory known to the HIP runtime", what);
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(TS_E_PLACEMENT, "%s: pointer is not device memory (memory type %d)", what,
                static_cast<int>(attr.type));
  if (attr.device != device)
    return fail(TS_E_PLACEMENT, "%s: pointer lives on device %d, the target is device %d", what, attr.device,
                device);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, const_cast<void*>(ptr));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TS_E_PLACEMENT, "%s: the allocation holding the pointer is unknown to the HIP runtime", what);
  }
  const uintptr_t p = reinterpret_cast<uintptr_t>(ptr);
  const uintptr_t lo = reinterpret_cast<uintptr_t>(base);
  const uint64_t room = (lo + size - p) / es;  // whole elements from ptr to the allocation's end
  if (n > room)
    return fail(TS_E_SHAPE, "%s: %llu elements from the pointer run past the end of its allocation (room for %llu)",
                what, static_cast<unsigned long long>(n), static_cast<unsigned long long>(room));
  return TS_OK;
}

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
  grid = cap_grid(grid, block);  // the loop strides over the rest
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
  log_choice(op, x->dtype, count, cls, 0, cfg);
  return launch_map(t, op, x->dtype, x->ptr, has_y ? y->ptr : nullptr, d->ptr, count, q, cfg);
}

void log_choice(int op, int dtype, uint64_t n, int align, int batched, const ts_kernel_cfg& c) {
  static const bool enabled = [] {
    const char* v = std::getenv("TS_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  if (!enabled) return;
  static std::mutex mu;
  static std::set<std::tuple<int, int, int, int, int>> seen;
  const int bucket = n ? 63 - __builtin_clzll(n) : 0;
  std::lock_guard<std::mutex> lk(mu);
  if (!seen.insert(std::make_tuple(op, dtype, bucket, align, batched)).second) return;
  static const char* const kOps[] = {"copy", "scale", "add", "triad"};
  static const char* const kTypes[] = {"f64", "f32", "bf16", "f16", "u8"};
  std::fprintf(stderr,
               "tstream: %s %s %s n=2^%d align=%d -> block %d, unroll %d, vec %d B, nt load %d, nt store %d, "
               "grid/CU %d, tile %lld x %d per workgroup\n",
               batched ? "batched" : "plain", kOps[op & 3], kTypes[dtype < 5 ? dtype : 0], bucket, align, c.block,
               c.unroll, c.vec_bytes, c.nt_load, c.nt_store, c.grid_per_cu, static_cast<long long>(c.tile_elems),
               c.tiles_per_wg < 1 ? 1 : c.tiles_per_wg);
}

}  // namespace tsapi

using namespace tsapi;

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
  // Set-up of the allocation-free checksum on this device (current here):
  // resolve its fixed array's address once, so later calls only look it up.
  CsPart* fixed_parts = nullptr;
  hipError_t e = noalloc_parts(device, &fixed_parts);
  if (e == hipSuccess) e = hipMalloc(&t->scratch, kReduceScratchBytes);
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
  // NULL: a non-blocking stream of the library's own.  hipStreamLegacy: the
  // device's legacy default stream, kept as the null handle.
  if (!hip_stream) return create_target(device, nullptr, true, out);
  if (hip_stream == static_cast<void*>(hipStreamLegacy)) return create_target(device, nullptr, false, out);
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
  a->alive = std::make_shared<bool>(true);
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
    if ((st = check_device_range(t->device, dev_ptr, n, es, "array")) != TS_OK) return st;
  }
  ts_array_s* a = new ts_array_s();
  a->alive = std::make_shared<bool>(true);
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
  *a->alive = false;
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

static_assert(sizeof(ts_checksum_out) == sizeof(CsPart) && offsetof(ts_checksum_out, sum) == offsetof(CsPart, sum) &&
                  offsetof(ts_checksum_out, abs_dev_sum) == offsetof(CsPart, absdev) &&
                  offsetof(ts_checksum_out, max_abs_dev) == offsetof(CsPart, maxdev) &&
                  offsetof(ts_checksum_out, mismatches) == offsetof(CsPart, mism),
              "the reduction kernel stores its result straight into a ts_checksum_out");

int ts_checksum_noalloc(ts_target t, ts_array x, double expected, ts_checksum_out* dev_out) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !ok_array(x) || !dev_out) return fail(TS_E_INVALID, "invalid handle or NULL dev_out");
  if (t->host) return host_only_gpu("ts_checksum_noalloc");
  if (!map_dtype(x->dtype)) return fail(TS_E_UNSUPPORTED, "checksums take floating-point storage");
  if (x->device != t->device) return fail(TS_E_PLACEMENT, "array is not on the executor's device");
  if (reinterpret_cast<uintptr_t>(dev_out) % alignof(ts_checksum_out))
    return fail(TS_E_INVALID, "dev_out must be aligned to %zu bytes", alignof(ts_checksum_out));
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  // Pointer queries only: nothing here allocates.
  if ((st = check_device_range(t->device, dev_out, 1, sizeof(ts_checksum_out), "dev_out")) != TS_OK) return st;
  const uintptr_t xo = reinterpret_cast<uintptr_t>(x->ptr), o = reinterpret_cast<uintptr_t>(dev_out);
  const uint64_t xbytes = x->n * dtype_size(x->dtype);
  if (o < xo + xbytes && xo < o + sizeof(ts_checksum_out))
    return fail(TS_E_ALIAS, "dev_out overlaps the array being reduced");
  const uint32_t np = checksum_parts(x->dtype, x->n);
  if (np > kNoallocParts)
    return fail(TS_E_SHAPE, "the reduction needs %u parts; the fixed array holds %u", np, kNoallocParts);
  CsPart* parts = nullptr;
  hipError_t e = noalloc_parts(t->device, &parts);
  if (e != hipSuccess) return hip_fail(e, "address of the fixed checksum array");
  CsPart* res = reinterpret_cast<CsPart*>(dev_out);
  e = x->n == 0 ? launch_store_part(res, CsPart{0.0, 0.0, 0.0, 0ull}, t->stream)
                : launch_checksum_to(x->dtype, x->ptr, x->n, expected, parts, res, t->stream);
  if (e != hipSuccess) return hip_fail(e, "checksum kernel launch");
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

}  // extern "C"
