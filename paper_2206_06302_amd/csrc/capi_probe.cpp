// capi_probe.cpp -- the memory-system probe of the C ABI: one launch of a
// straight-line kernel with a chosen mix of 16- or 8-byte reads and writes
// (kern_probe.hip), the ceiling the STREAM maps are measured against.
#include <cstdint>

#include "capi_internal.hpp"

using namespace ts;
using namespace tsapi;

namespace {

bool ranges_overlap(uintptr_t a, uintptr_t b, uint64_t bytes) { return a < b + bytes && b < a + bytes; }

int check_operand(const ts_target_s* t, const ts_array_s* a, uint64_t bytes, const char* name) {
  if (!ok_array(a)) return fail(TS_E_INVALID, "probe: invalid handle for %s", name);
  if (a->device != t->device) return fail(TS_E_PLACEMENT, "probe: %s is not on the executor's device", name);
  if (reinterpret_cast<uintptr_t>(a->ptr) % 16) return fail(TS_E_SHAPE, "probe: %s is not 16-byte aligned", name);
  if (a->n > UINT64_MAX / dtype_size(a->dtype) || a->n * dtype_size(a->dtype) < bytes)
    return fail(TS_E_SHAPE, "probe: %s holds fewer than %llu bytes", name, static_cast<unsigned long long>(bytes));
  return TS_OK;
}

}  // namespace

extern "C" {

int ts_probe_bandwidth(ts_target t, const ts_probe_cfg* cfg, ts_array x, ts_array y, ts_array dst, size_t bytes,
                       uint32_t mark) {
  TS_GUARD_BEGIN
  if (!ok_target(t) || !cfg) return fail(TS_E_INVALID, "probe: invalid target or NULL configuration");
  if (t->host) return fail(TS_E_UNSUPPORTED, "probe: GPU targets only");
  const ts_probe_cfg c = *cfg;
  if (c.reads < 0 || c.reads > 2 || c.writes < 0 || c.writes > 1 || c.reads + c.writes < 1)
    return fail(TS_E_INVALID, "probe: reads must be 0..2 and writes 0..1, not both 0");
  if (c.block < 64 || c.block > 1024 || c.block % 64)
    return fail(TS_E_INVALID, "probe: block must be 64..1024, a multiple of 64");
  if (c.unroll != 1 && c.unroll != 2 && c.unroll != 4) return fail(TS_E_INVALID, "probe: unroll must be 1, 2 or 4");
  if ((c.nt_load & ~1) || (c.nt_store & ~1) || (c.wave_contiguous & ~1))
    return fail(TS_E_INVALID, "probe: flags must be 0 or 1");
  if (c.vec_bytes != 0 && c.vec_bytes != 8 && c.vec_bytes != 16)
    return fail(TS_E_INVALID, "probe: vec_bytes must be 16 or 8 (0 means 16)");
  const uint64_t vb = c.vec_bytes ? static_cast<uint64_t>(c.vec_bytes) : 16u;
  int st = use_device(t->device);
  if (st != TS_OK) return st;
  int lds_per_cu = 0;
  TS_HIP(hipDeviceGetAttribute(&lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, t->device));
  if (c.lds_bytes < 0 || c.lds_bytes > lds_per_cu)
    return fail(TS_E_INVALID, "probe: lds_bytes must be 0..%d", lds_per_cu);
  const uint64_t per_wg = vb * static_cast<uint64_t>(c.block) * static_cast<uint64_t>(c.unroll);
  if (bytes == 0 || bytes % per_wg)
    return fail(TS_E_SHAPE, "probe: bytes must be a positive multiple of vec_bytes * block * unroll = %llu",
                static_cast<unsigned long long>(per_wg));
  const uint64_t grid = bytes / per_wg;
  if (grid > kMaxGridX) return fail(TS_E_SHAPE, "probe: more than 2^31 - 1 workgroups");
  if (grid * static_cast<uint64_t>(c.block) > kMaxWorkItems)
    return fail(TS_E_SHAPE, "probe: more than 2^32 - 1 lanes in one launch");
  if ((st = check_operand(t, dst, bytes, "dst")) != TS_OK) return st;
  const uintptr_t dp = reinterpret_cast<uintptr_t>(dst->ptr);
  if (c.reads >= 1) {
    if ((st = check_operand(t, x, bytes, "x")) != TS_OK) return st;
    if (ranges_overlap(reinterpret_cast<uintptr_t>(x->ptr), dp, bytes))
      return fail(TS_E_ALIAS, "probe: dst overlaps x");
  }
  if (c.reads == 2) {
    if ((st = check_operand(t, y, bytes, "y")) != TS_OK) return st;
    if (ranges_overlap(reinterpret_cast<uintptr_t>(y->ptr), dp, bytes))
      return fail(TS_E_ALIAS, "probe: dst overlaps y");
  }
  ProbeLaunch L{};
  L.x = c.reads >= 1 ? x->ptr : dst->ptr;
  L.y = c.reads == 2 ? y->ptr : L.x;
  L.d = dst->ptr;
  L.grid = static_cast<uint32_t>(grid);
  L.block = static_cast<uint32_t>(c.block);
  L.lds_bytes = static_cast<uint32_t>(c.lds_bytes);
  L.mark = mark;
  L.reads = c.reads;
  L.writes = c.writes;
  L.unroll = c.unroll;
  L.vb = static_cast<int>(vb);
  L.ntl = c.nt_load;
  L.nts = c.nt_store;
  L.wave_contiguous = c.wave_contiguous;
  L.stream = t->stream;
  const hipError_t e = launch_probe(L);
  if (e != hipSuccess) return hip_fail(e, "probe kernel launch");
  return TS_OK;
  TS_GUARD_END
}

}  // extern "C"
