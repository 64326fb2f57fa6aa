// ts_internal.hpp -- declarations shared by the host runtime and the kernel
// translation units of libtstream (not part of the public ABI).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "ts_layout.hpp"

namespace ts {

// Arguments of one plain launch: element-wise head, nvec vectors of vb
// bytes, element-wise tail (see plan_plain), and the launch shape.
struct PlainLaunch {
  const void* x;
  const void* y;
  void* d;
  double q;
  float qf;
  uint64_t head, nvec, tail;
  uint32_t grid, block;
  int op, vb, unroll, ntl, nts;
  hipStream_t stream;
};

// Arguments of one batched launch over a tile table.
struct BatchLaunch {
  const BatchTile* tiles;
  uint64_t ntiles;
  uint32_t grid, block;
  int op, unroll, ntl, nts;
  int tiles_per_wg;  // consecutive tiles per workgroup: 1, 2, 4 or 8
  int record_ahead;  // one workgroup per tile: read the record kRecordAhead ahead
  int pieces_log2;   // > 0: 2^pieces_log2 one-wave workgroups share each tile
  int vb;            // with pieces: bytes per lane access, 16 or 8
  hipStream_t stream;
};

// Arguments of one memory-system probe launch (kern_probe.hip): grid * block
// * unroll vectors of vb (16 or 8) bytes of each array involved.
struct ProbeLaunch {
  const void* x;
  const void* y;
  void* d;
  uint32_t grid, block, lds_bytes, mark;
  int reads, writes, unroll, vb, ntl, nts, wave_contiguous;
  hipStream_t stream;
};
hipError_t launch_probe(const ProbeLaunch& L);

// Per-format dispatch of the STREAM kernels (kern_<fmt>.hip).
hipError_t plain_launch_f64(const PlainLaunch& L);
hipError_t plain_launch_f32(const PlainLaunch& L);
hipError_t plain_launch_bf16(const PlainLaunch& L);
hipError_t plain_launch_f16(const PlainLaunch& L);
hipError_t batch_launch_f64(const BatchLaunch& L);
hipError_t batch_launch_f32(const BatchLaunch& L);
hipError_t batch_launch_bf16(const BatchLaunch& L);
hipError_t batch_launch_f16(const BatchLaunch& L);

// Partial results of the validation reductions (kern_aux.hip).
struct CsPart {
  double sum;
  double absdev;
  double maxdev;
  unsigned long long mism;
};

// Fixed reduction shape: depends only on n (and the address modulo 16
// bytes), never on tuning.
constexpr uint32_t kReduceBlock = 256;
constexpr uint32_t kReduceMaxParts = 8192;
// The first passes of the checksum and the mismatch count read chunks of
// kSumChunk 16-byte vectors (four per lane); one part per chunk, at most
// kSumMaxParts.
constexpr uint32_t kSumUnroll = 4;
constexpr uint64_t kSumChunk = static_cast<uint64_t>(kReduceBlock) * kSumUnroll;
constexpr uint32_t kSumMaxParts = 4096;
uint32_t checksum_parts(int dt, uint64_t n);
// Device scratch a target needs for one reduction: parts plus the result.
constexpr size_t kReduceScratchBytes = (kReduceMaxParts + 1) * sizeof(CsPart);

// Parts held by the fixed per-GPU array of the allocation-free checksum: as
// many as a checksum of any length uses, so it never limits n.
constexpr uint32_t kNoallocParts = kSumMaxParts;
// Devices whose fixed array's address is cached.
constexpr int kMaxDevices = 64;

// The constant fill's chunk: 256 lanes x two 8-byte words.
constexpr uint64_t kFillChunkWords = 512;
hipError_t launch_fill_const(int dt, void* p, uint64_t n, double value, hipStream_t s);
// Element j: lo + w * u01(first_index + j + 1), narrowed to the storage type.
hipError_t launch_fill_uniform(int dt, void* p, uint64_t n, uint64_t seed, uint64_t stream_id,
                               uint64_t first_index, double lo, double w, hipStream_t s);
// Leaves the reduced CsPart at scratch + kReduceMaxParts parts.
hipError_t launch_checksum(int dt, const void* x, uint64_t n, double expected, void* scratch,
                           hipStream_t s);
// The same two passes with the parts and the result wherever the caller says.
hipError_t launch_checksum_to(int dt, const void* x, uint64_t n, double expected, CsPart* parts, CsPart* out,
                              hipStream_t s);
// One kernel that stores v at *out (the result of an empty reduction).
hipError_t launch_store_part(CsPart* out, const CsPart& v, hipStream_t s);
// Device address, on `device`, of the allocation-free checksum's fixed array
// of kNoallocParts parts.  Resolved once per device; `device` must be the
// calling thread's current device on that first call.  Allocates nothing.
hipError_t noalloc_parts(int device, CsPart** out);
// Leaves the count in the `mism` field of the part after kReduceMaxParts.
hipError_t launch_mismatch(int dt, const void* x, const void* ref, uint64_t n, void* scratch,
                           hipStream_t s);
// Batched fills and mismatch counts give `per_wg` consecutive tiles to each
// workgroup of `grid` (which strides over any tiles beyond), kAuxBlock lanes
// per workgroup.
constexpr uint32_t kAuxBlock = 256;
// The most tiles one workgroup of those kernels takes: the records of a group
// are read together, so a workgroup waits on the table once per group.
constexpr uint32_t kAuxMaxTilesPerWg = 4;
hipError_t launch_batch_fill(int dt, const BatchTile* tiles, uint64_t ntiles, uint32_t per_wg, int which,
                             int uniform, double value, uint64_t seed, uint32_t grid, hipStream_t s);
// counts: device array of one unsigned long long per instance, zeroed by the
// caller's fill kernel (launch_zero_u64).
hipError_t launch_batch_mismatch(int dt, const BatchTile* tiles, uint64_t ntiles, uint32_t per_wg, int which,
                                 const double* expected, unsigned long long* counts, uint32_t grid,
                                 hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, uint64_t n, hipStream_t s);

}  // namespace ts
