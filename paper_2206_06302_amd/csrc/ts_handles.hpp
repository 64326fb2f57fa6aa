// ts_handles.hpp -- definitions of the target and array handles of
// libtstream, shared by the translation units that implement the C ABI (not
// part of the public interface).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <memory>

#include "../../include/tstream.h"
#include "host_target.hpp"

namespace ts {
constexpr uint32_t kTargetMagic = 0x54475431u;  // "TGT1"
constexpr uint32_t kArrayMagic = 0x41525231u;

// Record a failure message for ts_last_error() and return `status`.
int api_fail(int status, const char* fmt, ...);
// Map a HIP error to TS_E_OOM / TS_E_DEVICE with its text.
int api_hip_fail(hipError_t e, const char* what);
}  // namespace ts

struct ts_target_s {
  uint32_t magic;
  int device;  // -1 for a host-CPU target
  bool host;
  ts::HostPool* pool;  // host targets: the pinned workers
  hipStream_t stream;
  bool owns_stream;
  ts_device_info info;
  void* scratch;  // reduction parts + result (kReduceScratchBytes)
  void* host_result;
};

struct ts_array_s {
  uint32_t magic;
  ts_target_s* target;
  int device;  // -1: host memory of a host target
  int dtype;
  void* ptr;
  uint64_t n;
  void* owned_base;
  // Cleared by ts_array_free; graphs captured over the array share it and
  // refuse to launch once it is cleared.
  std::shared_ptr<bool> alive;
};

inline bool ts_ok_target_handle(const ts_target_s* t) { return t && t->magic == ts::kTargetMagic; }
inline bool ts_ok_array_handle(const ts_array_s* a) { return a && a->magic == ts::kArrayMagic; }
