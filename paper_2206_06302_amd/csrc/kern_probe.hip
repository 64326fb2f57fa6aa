// kern_probe.hip -- memory-system probe kernels: straight-line 16- or
// 8-byte vector traffic with each mix of reads and writes, and no arithmetic
// beyond a bitwise fold.  They measure what the memory system delivers for
// read-only, write-only, one-read-one-write and two-reads-one-write streams,
// the ceilings against which the STREAM maps (copy and scale: one read, one
// write; add and triad: two reads, one write) are judged, in the same access
// widths the maps use.  They are measurement tools, not one of the paper's
// algorithms.
#include "ts_device.hpp"
#include "ts_internal.hpp"

namespace ts {

namespace {

template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT, typename V>
__device__ __forceinline__ void st(V* p, V v) {
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

// Every 32-bit word of a vector set to m.
template <typename V>
__device__ __forceinline__ V splat(uint32_t m) {
  V v;
#pragma unroll
  for (int i = 0; i < static_cast<int>(sizeof(V) / 4); ++i) v[i] = m;
  return v;
}

// R arrays read (x, then y), W arrays written (d), VB-byte vectors.  With
// W = 1: d = x (R = 1), d = x ^ y (R = 2) or d = the mark pattern (R = 0).
// With W = 0 every lane folds what it reads and stores the fold at d[lane's
// global index] only if its first word equals `mark`, which keeps the loads
// alive.
template <int VB, int R, int W, int U, bool NTL, bool NTS, bool WAVE>
__global__ __launch_bounds__(1024) void probe_kernel(const typename Raw<VB>::type* __restrict__ x,
                                                     const typename Raw<VB>::type* __restrict__ y,
                                                     typename Raw<VB>::type* __restrict__ d, uint32_t mark) {
  using V = typename Raw<VB>::type;
  V a[U], b[U];
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
      V o;
      if constexpr (R == 0) o = splat<V>(mark);
      else if constexpr (R == 1) o = a[k];
      else o = a[k] ^ b[k];
      st<NTS>(d + v, o);
    }
  } else {
    V f = splat<V>(0u);
#pragma unroll
    for (int k = 0; k < U; ++k) {
      f ^= a[k];
      if constexpr (R == 2) f ^= b[k];
    }
    if (f.x == mark) d[static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = f;
  }
}

template <int VB, int R, int W, int U, bool NTL, bool NTS, bool WAVE>
hipError_t launch_inst(const ProbeLaunch& L) {
  using V = typename Raw<VB>::type;
  auto kern = probe_kernel<VB, R, W, U, NTL, NTS, WAVE>;
  if (L.lds_bytes > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(L.lds_bytes));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.block), L.lds_bytes, L.stream, static_cast<const V*>(L.x),
                     static_cast<const V*>(L.y), static_cast<V*>(L.d), L.mark);
  return hipGetLastError();
}

template <int VB, int R, int W, int U, bool NTL, bool NTS>
hipError_t by_layout(const ProbeLaunch& L) {
  return L.wave_contiguous ? launch_inst<VB, R, W, U, NTL, NTS, true>(L)
                           : launch_inst<VB, R, W, U, NTL, NTS, false>(L);
}

template <int VB, int R, int W, int U>
hipError_t by_nt(const ProbeLaunch& L) {
  if (L.ntl) return L.nts ? by_layout<VB, R, W, U, true, true>(L) : by_layout<VB, R, W, U, true, false>(L);
  return L.nts ? by_layout<VB, R, W, U, false, true>(L) : by_layout<VB, R, W, U, false, false>(L);
}

template <int VB, int R, int W>
hipError_t by_unroll(const ProbeLaunch& L) {
  switch (L.unroll) {
    case 1: return by_nt<VB, R, W, 1>(L);
    case 2: return by_nt<VB, R, W, 2>(L);
    case 4: return by_nt<VB, R, W, 4>(L);
    default: return hipErrorInvalidValue;
  }
}

template <int R, int W>
hipError_t by_width(const ProbeLaunch& L) {
  switch (L.vb) {
    case 16: return by_unroll<16, R, W>(L);
    case 8: return by_unroll<8, R, W>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_probe(const ProbeLaunch& L) {
  if (L.reads == 1 && L.writes == 0) return by_width<1, 0>(L);
  if (L.reads == 2 && L.writes == 0) return by_width<2, 0>(L);
  if (L.reads == 0 && L.writes == 1) return by_width<0, 1>(L);
  if (L.reads == 1 && L.writes == 1) return by_width<1, 1>(L);
  if (L.reads == 2 && L.writes == 1) return by_width<2, 1>(L);
  return hipErrorInvalidValue;
}

}  // namespace ts
