// kern_probe.hip -- memory-system probe kernels: straight-line 16-byte vector
// traffic with each mix of reads and writes, and no arithmetic beyond a
// bitwise fold.  They measure what the memory system delivers for read-only,
// write-only, one-read-one-write and two-reads-one-write streams, the
// ceilings against which the STREAM maps (copy and scale: one read, one
// write; add and triad: two reads, one write) are judged.  They are
// measurement tools, not one of the paper's algorithms.
#include "ts_device.hpp"
#include "ts_internal.hpp"

namespace ts {

namespace {

using V4 = Raw<16>::type;

template <bool NT>
__device__ __forceinline__ V4 ld(const V4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT>
__device__ __forceinline__ void st(V4* p, V4 v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Workgroup w covers vectors [w*B*U, (w+1)*B*U) of every array (B lanes, U
// vectors per lane).  Block-strided: a lane's vectors lie B apart, so every
// step of the workgroup covers B consecutive vectors.  Wave-contiguous: wave
// k covers U*64 consecutive vectors, a lane's vectors lie 64 apart.
template <int U, bool WAVE>
__device__ __forceinline__ uint64_t vec_index(int k) {
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * blockDim.x * U;
  if constexpr (WAVE) {
    const uint64_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    return base + wave * 64 * U + static_cast<uint64_t>(k) * 64 + lane;
  } else {
    return base + static_cast<uint64_t>(k) * blockDim.x + threadIdx.x;
  }
}

// R arrays read (x, then y), W arrays written (d).  With W = 1: d = x
// (R = 1), d = x ^ y (R = 2) or d = the mark pattern (R = 0).  With W = 0
// every lane folds what it reads and stores the fold at d[lane's global
// index] only if its first word equals `mark`, which keeps the loads alive.
template <int R, int W, int U, bool NTL, bool NTS, bool WAVE>
__global__ __launch_bounds__(1024) void probe_kernel(const V4* __restrict__ x, const V4* __restrict__ y,
                                                     V4* __restrict__ d, uint32_t mark) {
  V4 a[U], b[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const uint64_t v = vec_index<U, WAVE>(k);
    if constexpr (R >= 1) a[k] = ld<NTL>(x + v);
    if constexpr (R == 2) b[k] = ld<NTL>(y + v);
  }
  if constexpr (W == 1) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint64_t v = vec_index<U, WAVE>(k);
      V4 o;
      if constexpr (R == 0) o = V4{mark, mark, mark, mark};
      else if constexpr (R == 1) o = a[k];
      else o = a[k] ^ b[k];
      st<NTS>(d + v, o);
    }
  } else {
    V4 f = V4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < U; ++k) {
      f ^= a[k];
      if constexpr (R == 2) f ^= b[k];
    }
    if (f.x == mark) d[static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = f;
  }
}

template <int R, int W, int U, bool NTL, bool NTS, bool WAVE>
hipError_t launch_inst(const ProbeLaunch& L) {
  auto kern = probe_kernel<R, W, U, NTL, NTS, WAVE>;
  if (L.lds_bytes > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(L.lds_bytes));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.block), L.lds_bytes, L.stream,
                     static_cast<const V4*>(L.x), static_cast<const V4*>(L.y), static_cast<V4*>(L.d), L.mark);
  return hipGetLastError();
}

template <int R, int W, int U, bool NTL, bool NTS>
hipError_t by_layout(const ProbeLaunch& L) {
  return L.wave_contiguous ? launch_inst<R, W, U, NTL, NTS, true>(L) : launch_inst<R, W, U, NTL, NTS, false>(L);
}

template <int R, int W, int U>
hipError_t by_nt(const ProbeLaunch& L) {
  if (L.ntl) return L.nts ? by_layout<R, W, U, true, true>(L) : by_layout<R, W, U, true, false>(L);
  return L.nts ? by_layout<R, W, U, false, true>(L) : by_layout<R, W, U, false, false>(L);
}

template <int R, int W>
hipError_t by_unroll(const ProbeLaunch& L) {
  switch (L.unroll) {
    case 1: return by_nt<R, W, 1>(L);
    case 2: return by_nt<R, W, 2>(L);
    case 4: return by_nt<R, W, 4>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_probe(const ProbeLaunch& L) {
  if (L.reads == 1 && L.writes == 0) return by_unroll<1, 0>(L);
  if (L.reads == 2 && L.writes == 0) return by_unroll<2, 0>(L);
  if (L.reads == 0 && L.writes == 1) return by_unroll<0, 1>(L);
  if (L.reads == 1 && L.writes == 1) return by_unroll<1, 1>(L);
  if (L.reads == 2 && L.writes == 1) return by_unroll<2, 1>(L);
  return hipErrorInvalidValue;
}

}  // namespace ts
