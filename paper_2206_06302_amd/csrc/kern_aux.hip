// kern_aux.hip -- device-side bulk construction (fill) and the validation
// reductions used to check STREAM results on the GPU.
//
// Bulk construction runs on the device, as the paper's GPU allocator does
// (Section 3.2, Listing 1's bulk_construct; Section 4.2).  The uniform fill
// is SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) evaluated at a counter,
// so any element can be regenerated alone.
#include <cmath>
#include <mutex>

#include "ts_device.hpp"
#include "ts_internal.hpp"

namespace ts {

// Reduction parts of the allocation-free checksum (ts_checksum_noalloc): one
// fixed array per GPU, loaded with the library's code object and held until
// the process ends.  Host code never passes this name to a kernel (on the
// host it is only a stand-in for the symbol); it resolves the array's
// device address once per device (noalloc_parts) and passes that.
static __device__ __align__(256) CsPart noalloc_scratch[kNoallocParts];

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Store a binary64 value into storage format DT: binary32 by nearest-even,
// then the 16-bit formats by nearest-even from that binary32 value.
template <int DT>
__device__ __forceinline__ typename Fmt<DT>::T from_f64(double v) {
  if constexpr (DT == DT_F64) return v;
  else if constexpr (DT == DT_F32) return static_cast<float>(v);
  else return narrow<DT>(static_cast<float>(v));
}

template <int DT>
__device__ __forceinline__ double to_f64(typename Fmt<DT>::T v) {
  return static_cast<double>(widen<DT>(v));
}

__device__ __forceinline__ double uniform_pm1(uint64_t state0, uint64_t counter) {
  const uint64_t h = splitmix64_mix(state0 + counter * kGamma);
  return static_cast<double>(h >> 11) * 0x1p-52 - 1.0;
}

__device__ __forceinline__ bool differs(double v, double e) {
  if (__builtin_isnan(v) && __builtin_isnan(e)) return false;
  return __builtin_bit_cast(uint64_t, v) != __builtin_bit_cast(uint64_t, e);
}

// 16 bytes of one repeated element.
template <class T>
struct Splat {
  T e[16 / sizeof(T)];
};

// 8 bytes of one repeated element.
template <class T>
struct Splat8 {
  T e[8 / sizeof(T)];
};

// Elements [0, head) and those after the `nwords` 8-byte words are stored one
// by one.  The words in between go in chunks of kFillChunkWords (4 KiB), chunk
// c to workgroup c modulo the grid: each of its four waves stores one
// contiguous KiB with two 8-byte nontemporal stores per lane.
template <int DT>
__global__ __launch_bounds__(256) void fill_const_kernel(void* p, uint64_t n, double value, uint64_t head,
                                                         uint64_t nwords) {
  using T = typename Fmt<DT>::T;
  using W = typename Raw<8>::type;
  constexpr uint64_t E = 8 / sizeof(T);
  T* d = static_cast<T*>(p);
  const T v = from_f64<DT>(value);
  const uint32_t t = threadIdx.x;
  const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + t;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t j = g; j < head; j += stride) d[j] = v;
  for (uint64_t j = head + nwords * E + g; j < n; j += stride) d[j] = v;
  Splat8<T> s;
#pragma unroll
  for (uint64_t e = 0; e < E; ++e) s.e[e] = v;
  const W r = __builtin_bit_cast(W, s);
  W* dw = reinterpret_cast<W*>(d + head);
  const uint64_t lane_word = (t >> 6) * 128 + (t & 63);
  for (uint64_t c = blockIdx.x; c * kFillChunkWords < nwords; c += gridDim.x) {
    const uint64_t i = c * kFillChunkWords + lane_word;
    if (i < nwords) __builtin_nontemporal_store(r, dw + i);
    if (i + 64 < nwords) __builtin_nontemporal_store(r, dw + i + 64);
  }
}

// lo + w * u01 with u01 = (h >> 11) * 2^-53 in [0, 1): a product and a sum,
// each rounded (nothing is contracted).  For lo = -1, w = 2 every step is
// exact and the value equals uniform_pm1's.
__device__ __forceinline__ double uniform_range(uint64_t state0, uint64_t counter, double lo, double w) {
  const uint64_t h = splitmix64_mix(state0 + counter * kGamma);
  return lo + w * (static_cast<double>(h >> 11) * 0x1p-53);
}

// Element j gets counter first + j + 1; the layout (head, 16-byte vectors,
// tail) is that of fill_const_kernel and does not change any value.
template <int DT>
__global__ __launch_bounds__(256) void fill_uniform_kernel(void* p, uint64_t n, uint64_t state0,
                                                           uint64_t first, double lo, double w, uint64_t head,
                                                           uint64_t nvec) {
  using T = typename Fmt<DT>::T;
  using R = typename Raw<16>::type;
  constexpr uint64_t E = 16 / sizeof(T);
  T* d = static_cast<T*>(p);
  const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  auto value = [&](uint64_t j) { return from_f64<DT>(uniform_range(state0, first + j + 1, lo, w)); };
  for (uint64_t j = g; j < head; j += stride) d[j] = value(j);
  for (uint64_t j = head + nvec * E + g; j < n; j += stride) d[j] = value(j);
  R* dv = reinterpret_cast<R*>(d + head);
  for (uint64_t k = g; k < nvec; k += stride) {
    Splat<T> s;
#pragma unroll
    for (uint64_t e = 0; e < E; ++e) s.e[e] = value(head + k * E + e);
    __builtin_nontemporal_store(__builtin_bit_cast(R, s), dv + k);
  }
}

__device__ __forceinline__ void combine(CsPart& a, const CsPart& b) {
  a.sum += b.sum;
  a.absdev += b.absdev;
  a.maxdev = fmax(a.maxdev, b.maxdev);
  a.mism += b.mism;
}

// Fixed-order tree over the 256 lanes of a workgroup.
__device__ CsPart block_reduce(CsPart v) {
  __shared__ double s_sum[kReduceBlock], s_abs[kReduceBlock], s_max[kReduceBlock];
  __shared__ unsigned long long s_cnt[kReduceBlock];
  const uint32_t t = threadIdx.x;
  s_sum[t] = v.sum;
  s_abs[t] = v.absdev;
  s_max[t] = v.maxdev;
  s_cnt[t] = v.mism;
  __syncthreads();
  for (uint32_t s = kReduceBlock / 2; s > 0; s >>= 1) {
    if (t < s) {
      s_sum[t] += s_sum[t + s];
      s_abs[t] += s_abs[t + s];
      s_max[t] = fmax(s_max[t], s_max[t + s]);
      s_cnt[t] += s_cnt[t + s];
    }
    __syncthreads();
  }
  return CsPart{s_sum[0], s_abs[0], s_max[0], s_cnt[0]};
}

// Split the range [lo, hi) of `x` into an element-wise head up to the next
// 16-byte boundary, whole 16-byte vectors, and an element-wise tail (both
// shorter than one vector).  `x` is aligned to its element size.
template <class T>
struct VecRange {
  uint64_t head, v0, nvec, t0;  // head elements at lo; vectors from v0; tail from t0 to hi
};

template <class T>
__device__ __forceinline__ VecRange<T> vec_range(const T* x, uint64_t lo, uint64_t hi) {
  constexpr uint64_t E = 16 / sizeof(T);
  const uint64_t mis = reinterpret_cast<uintptr_t>(x + lo) % 16;
  uint64_t head = ((16 - mis) % 16) / sizeof(T);
  if (head > hi - lo) head = hi - lo;
  const uint64_t v0 = lo + head;
  const uint64_t nvec = (hi - v0) / E;
  return VecRange<T>{head, v0, nvec, v0 + nvec * E};
}

// Pass 1: the 16-byte vectors of x form chunks of kSumChunk vectors (four per
// lane); workgroup g of G folds chunks g, g + G, g + 2G, ... with nontemporal
// loads, the next chunk's loads issued before the current chunk is folded.
// Workgroup 0 also folds the element-wise head before the first vector and
// the tail after the last.  Each lane folds its elements in ascending order,
// so the tree depends only on n, the storage type and the array's address
// modulo 16 bytes.  An element is a mismatch when its binary64 bits differ
// from expected's, two NaNs agreeing (differs); EM, chosen per launch from
// `expected`, gives that test its cheapest exact form: kExpNan (expected is
// a NaN: the element is not one), kExpZero (expected is +0 or -0: compare the
// bits) or kExpValue (any other expected: compare the values, since a
// nonzero binary64 value has one encoding and a NaN compares unequal).
enum : int { kExpValue = 0, kExpNan = 1, kExpZero = 2 };
template <int DT, int EM>
__global__ __launch_bounds__(256) void checksum_pass1(const void* xv, uint64_t n, double expected,
                                                      CsPart* parts, uint32_t nparts) {
  using T = typename Fmt<DT>::T;
  using R = typename Raw<16>::type;
  constexpr uint32_t E = 16 / sizeof(T);
  const T* x = static_cast<const T*>(xv);
  const uint32_t t = threadIdx.x;
  CsPart acc{0.0, 0.0, __builtin_nan(""), 0ull};
  uint32_t mism = 0;  // a lane folds far fewer than 2^32 elements
  auto add = [&](double v) {
    const double dv = fabs(v - expected);
    acc.sum += v;
    acc.absdev += dv;
    acc.maxdev = fmax(acc.maxdev, dv);
    bool d;
    if constexpr (EM == kExpNan) d = !__builtin_isnan(v);
    else if constexpr (EM == kExpZero) d = __builtin_bit_cast(uint64_t, v) != __builtin_bit_cast(uint64_t, expected);
    else d = v != expected;
    mism += d ? 1u : 0u;
  };
  auto fold = [&](R r) {
    if constexpr (sizeof(T) == 2) {
      // Two elements per 32-bit word, the lower address in the low half.
#pragma unroll
      for (uint32_t w = 0; w < 4; ++w) {
        const uint32_t b = r[w];
        if constexpr (DT == DT_BF16) {
          add(static_cast<double>(__builtin_bit_cast(float, b << 16)));
          add(static_cast<double>(__builtin_bit_cast(float, b & 0xffff0000u)));
        } else {
          add(to_f64<DT>(static_cast<uint16_t>(b)));
          add(to_f64<DT>(static_cast<uint16_t>(b >> 16)));
        }
      }
    } else {
      const Splat<T> v = __builtin_bit_cast(Splat<T>, r);
#pragma unroll
      for (uint32_t e = 0; e < E; ++e) add(to_f64<DT>(v.e[e]));
    }
  };
  const VecRange<T> vr = vec_range(x, 0, n);
  if (blockIdx.x == 0 && t < vr.head) add(to_f64<DT>(x[t]));
  const R* xr = reinterpret_cast<const R*>(x + vr.v0);
  const uint64_t nvec = vr.nvec, step = static_cast<uint64_t>(nparts) * kSumChunk;
  uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSumChunk;
  if (base + kSumChunk <= nvec) {
    R cur[kSumUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kSumUnroll; ++u) cur[u] = __builtin_nontemporal_load(xr + base + u * kReduceBlock + t);
    for (base += step; base + kSumChunk <= nvec; base += step) {
      R nxt[kSumUnroll];
#pragma unroll
      for (uint32_t u = 0; u < kSumUnroll; ++u) nxt[u] = __builtin_nontemporal_load(xr + base + u * kReduceBlock + t);
#pragma unroll
      for (uint32_t u = 0; u < kSumUnroll; ++u) fold(cur[u]);
#pragma unroll
      for (uint32_t u = 0; u < kSumUnroll; ++u) cur[u] = nxt[u];
    }
#pragma unroll
    for (uint32_t u = 0; u < kSumUnroll; ++u) fold(cur[u]);
  }
  // The chunk cut short by the end of the vectors, if it is this workgroup's.
  for (uint64_t k = base + t; k < nvec; k += kReduceBlock) fold(__builtin_nontemporal_load(xr + k));
  if (blockIdx.x == 0 && t < n - vr.t0) add(to_f64<DT>(x[vr.t0 + t]));
  acc.mism = mism;
  const CsPart r = block_reduce(acc);
  if (t == 0) parts[blockIdx.x] = r;
}

// Pass 2: one workgroup folds the parts in a fixed order.
__global__ __launch_bounds__(256) void reduce_pass2(const CsPart* parts, uint32_t nparts, CsPart* out) {
  CsPart acc{0.0, 0.0, __builtin_nan(""), 0ull};
  uint32_t j = threadIdx.x;
  for (; j + 3 * kReduceBlock < nparts; j += 4 * kReduceBlock) {  // loads first, then the folds in order
    const CsPart p0 = parts[j], p1 = parts[j + kReduceBlock], p2 = parts[j + 2 * kReduceBlock],
                 p3 = parts[j + 3 * kReduceBlock];
    combine(acc, p0), combine(acc, p1), combine(acc, p2), combine(acc, p3);
  }
  for (; j < nparts; j += kReduceBlock) combine(acc, parts[j]);
  const CsPart r = block_reduce(acc);
  if (threadIdx.x == 0) *out = r;
}

// Count of elements whose bits differ between x and r (two NaNs agree).
// When x and r share their address modulo 16 bytes, their 16-byte vectors
// form chunks of kSumChunk vectors as in checksum_pass1: workgroup g of P
// counts chunks g, g + P, g + 2P, ..., issuing the next chunk's loads before
// it compares the current one, and workgroup 0 also the element-wise head
// and tail.  Otherwise workgroup g counts the contiguous range
// [g*n/P, (g+1)*n/P) element by element.  A count is a sum of integers, so
// the split does not change it.
template <int DT>
__global__ __launch_bounds__(256) void mismatch_pass1(const void* xv, const void* rv, uint64_t n,
                                                      CsPart* parts, uint32_t nparts) {
  using T = typename Fmt<DT>::T;
  using R = typename Raw<16>::type;
  constexpr uint32_t E = 16 / sizeof(T);
  const T* x = static_cast<const T*>(xv);
  const T* r = static_cast<const T*>(rv);
  const uint32_t t = threadIdx.x;
  CsPart acc{0.0, 0.0, 0.0, 0ull};
  uint32_t mism = 0;  // a lane compares far fewer than 2^32 elements
  auto count = [&](T a, T b) {
    bool diff;
    if constexpr (sizeof(T) == 8) diff = __builtin_bit_cast(uint64_t, a) != __builtin_bit_cast(uint64_t, b);
    else if constexpr (sizeof(T) == 4) diff = __builtin_bit_cast(uint32_t, a) != __builtin_bit_cast(uint32_t, b);
    else diff = a != b;
    if (diff && __builtin_isnan(to_f64<DT>(a)) && __builtin_isnan(to_f64<DT>(b))) diff = false;
    mism += diff ? 1u : 0u;
  };
  auto fold = [&](R ra, R rb) {
    const Splat<T> va = __builtin_bit_cast(Splat<T>, ra), vb = __builtin_bit_cast(Splat<T>, rb);
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) count(va.e[e], vb.e[e]);
  };
  if ((reinterpret_cast<uintptr_t>(x) - reinterpret_cast<uintptr_t>(r)) % 16 == 0) {
    const VecRange<T> vr = vec_range(x, 0, n);
    if (blockIdx.x == 0 && t < vr.head) count(x[t], r[t]);
    const R* xr = reinterpret_cast<const R*>(x + vr.v0);
    const R* rr = reinterpret_cast<const R*>(r + vr.v0);
    const uint64_t nvec = vr.nvec, step = static_cast<uint64_t>(nparts) * kSumChunk;
    uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSumChunk;
    if (base + kSumChunk <= nvec) {
      R ca[kSumUnroll], cb[kSumUnroll];
#pragma unroll
      for (uint32_t u = 0; u < kSumUnroll; ++u) {
        ca[u] = __builtin_nontemporal_load(xr + base + u * kReduceBlock + t);
        cb[u] = __builtin_nontemporal_load(rr + base + u * kReduceBlock + t);
      }
      for (base += step; base + kSumChunk <= nvec; base += step) {
        R na[kSumUnroll], nb[kSumUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kSumUnroll; ++u) {
          na[u] = __builtin_nontemporal_load(xr + base + u * kReduceBlock + t);
          nb[u] = __builtin_nontemporal_load(rr + base + u * kReduceBlock + t);
        }
#pragma unroll
        for (uint32_t u = 0; u < kSumUnroll; ++u) fold(ca[u], cb[u]);
#pragma unroll
        for (uint32_t u = 0; u < kSumUnroll; ++u) ca[u] = na[u], cb[u] = nb[u];
      }
#pragma unroll
      for (uint32_t u = 0; u < kSumUnroll; ++u) fold(ca[u], cb[u]);
    }
    // The chunk cut short by the end of the vectors, if it is this workgroup's.
    for (uint64_t k = base + t; k < nvec; k += kReduceBlock)
      fold(__builtin_nontemporal_load(xr + k), __builtin_nontemporal_load(rr + k));
    if (blockIdx.x == 0 && t < n - vr.t0) count(x[vr.t0 + t], r[vr.t0 + t]);
  } else {
    const uint64_t lo = static_cast<uint64_t>(blockIdx.x) * n / nparts;
    const uint64_t hi = static_cast<uint64_t>(blockIdx.x + 1) * n / nparts;
    uint64_t j = lo + t;
    for (; j + kReduceBlock < hi; j += 2 * kReduceBlock) {  // two pairs of loads in flight per lane
      const T a0 = x[j], b0 = r[j], a1 = x[j + kReduceBlock], b1 = r[j + kReduceBlock];
      count(a0, b0), count(a1, b1);
    }
    for (; j < hi; j += kReduceBlock) count(x[j], r[j]);
  }
  acc.mism = mism;
  const CsPart res = block_reduce(acc);
  if (t == 0) parts[blockIdx.x] = res;
}

// Whole 16-byte vectors [vs, ve) inside the tile [start, end) of an array
// whose first `h` elements come before its first 16-byte boundary.
__device__ __forceinline__ void tile_vectors(uint64_t start, uint64_t end, uint64_t h, uint64_t V,
                                             uint64_t& vs, uint64_t& ve) {
  vs = start < h ? h : h + (start - h + V - 1) / V * V;
  if (vs > end) vs = end;
  ve = end < h ? vs : h + (end - h) / V * V;
  if (ve < vs) ve = vs;
}

template <class T>
__device__ __forceinline__ uint64_t head_of(const T* p) {
  return ((16 - reinterpret_cast<uintptr_t>(p) % 16) % 16) / sizeof(T);
}

// Tiles [c, c + per_wg) of the table go to workgroup c / per_wg (striding
// by the grid over any beyond it), per_wg at most kAuxMaxTilesPerWg.  A
// workgroup reads the records of its group together (scalar loads issued
// back to back), so it waits on the table once per group, not once per tile.
#define TS_FOR_TILE_GROUPS(c0, cnt)                                                               \
  for (uint64_t c0 = static_cast<uint64_t>(blockIdx.x) * per_wg, cnt = 0; c0 < ntiles;             \
       c0 += static_cast<uint64_t>(gridDim.x) * per_wg)                                           \
    if ((cnt = ntiles - c0 < per_wg ? ntiles - c0 : per_wg), true)

// Tile by tile, for kernels that wait on each tile's data anyway.
#define TS_FOR_TILES(t)                                                                           \
  for (uint64_t c_ = static_cast<uint64_t>(blockIdx.x) * per_wg; c_ < ntiles;                    \
       c_ += static_cast<uint64_t>(gridDim.x) * per_wg)                                           \
    for (uint64_t t = c_, e_ = ntiles - c_ < per_wg ? ntiles : c_ + per_wg; t < e_; ++t)

// Fill one array of every instance (which: 0 a, 1 b, 2 c), tile by tile:
// elements before and after the tile's whole 16-byte vectors one per lane,
// the vectors with nontemporal stores.  Element j of instance i gets the
// constant (UNIFORM false), or uniform draw j + 1 of stream 16 + 3i + which.
// The tile table is read-only here, so its records are scalar loads.
template <int DT, bool UNIFORM>
__global__ __launch_bounds__(256) void batch_fill_kernel(const BatchTile* __restrict__ tiles,
                                                         uint64_t ntiles, uint32_t per_wg, int which,
                                                         double value, uint64_t seed) {
  using T = typename Fmt<DT>::T;
  using R = typename Raw<16>::type;
  constexpr uint64_t V = 16 / sizeof(T);
  TS_FOR_TILE_GROUPS(c0, cnt) {
    BatchTile group[kAuxMaxTilesPerWg];  // past the group's end: its last record again, unused
#pragma unroll
    for (uint32_t g = 0; g < kAuxMaxTilesPerWg; ++g) group[g] = tiles[c0 + (g < cnt ? g : cnt - 1)];
#pragma unroll
    for (uint32_t g = 0; g < kAuxMaxTilesPerWg; ++g) {
      if (g >= cnt) break;
      const BatchTile& tl = group[g];
      T* dp = static_cast<T*>(const_cast<void*>(which == 0 ? tl.a : which == 1 ? tl.b : tl.c));
      Global<T>* d = global_ptr(dp);  // global_load/store, not flat (see ts_device.hpp)
      const uint64_t state0 = seed ^ ((16ull + 3ull * tl.inst + static_cast<uint64_t>(which)) << 48);
      const T cv = from_f64<DT>(value);
      auto at = [&](uint64_t j) {
        if constexpr (UNIFORM) return from_f64<DT>(uniform_pm1(state0, j + 1));
        else return cv;
      };
      const uint64_t end = tl.start + tl.count;
      uint64_t vs, ve;
      tile_vectors(tl.start, end, head_of(dp), V, vs, ve);
      Global<R>* dv = reinterpret_cast<Global<R>*>(d + vs);
      const uint64_t nvec = (ve - vs) / V;
      for (uint64_t k = threadIdx.x; k < nvec; k += blockDim.x) {
        Splat<T> v;
#pragma unroll
        for (uint64_t e = 0; e < V; ++e) v.e[e] = at(vs + k * V + e);
        __builtin_nontemporal_store(__builtin_bit_cast(R, v), dv + k);
      }
      for (uint64_t j = tl.start + threadIdx.x; j < vs; j += blockDim.x) d[j] = at(j);
      for (uint64_t j = ve + threadIdx.x; j < end; j += blockDim.x) d[j] = at(j);
    }
  }
}

// Per-instance count of elements of one array whose binary64 value differs
// in bits from the instance's expected value, read like batch_fill_kernel
// writes.  Each lane counts its own elements of a tile and adds its count
// to the instance's counter only when it found a mismatch (integer adds, so
// the totals do not depend on their order).
template <int DT>
__global__ __launch_bounds__(256) void batch_mismatch_kernel(const BatchTile* __restrict__ tiles,
                                                             uint64_t ntiles, uint32_t per_wg, int which,
                                                             const double* __restrict__ expected,
                                                             unsigned long long* counts) {
  using T = typename Fmt<DT>::T;
  using R = typename Raw<16>::type;
  constexpr uint64_t V = 16 / sizeof(T);
  TS_FOR_TILES(t) {
    const BatchTile tl = tiles[t];
    const T* xp = static_cast<const T*>(which == 0 ? tl.a : which == 1 ? tl.b : tl.c);
    const Global<T>* x = global_ptr(xp);
    const double e = expected[tl.inst];
    const uint64_t end = tl.start + tl.count;
    uint64_t vs, ve;
    tile_vectors(tl.start, end, head_of(xp), V, vs, ve);
    unsigned long long c = 0;
    for (uint64_t j = tl.start + threadIdx.x; j < vs; j += blockDim.x) c += differs(to_f64<DT>(x[j]), e) ? 1 : 0;
    for (uint64_t j = ve + threadIdx.x; j < end; j += blockDim.x) c += differs(to_f64<DT>(x[j]), e) ? 1 : 0;
    const Global<R>* xv = reinterpret_cast<const Global<R>*>(x + vs);
    const uint64_t nvec = (ve - vs) / V;
    for (uint64_t k = threadIdx.x; k < nvec; k += blockDim.x) {
      const Splat<T> v = __builtin_bit_cast(Splat<T>, __builtin_nontemporal_load(xv + k));
#pragma unroll
      for (uint64_t i = 0; i < V; ++i) c += differs(to_f64<DT>(v.e[i]), e) ? 1 : 0;
    }
    if (c) atomicAdd(&counts[tl.inst], c);
  }
}

__global__ __launch_bounds__(256) void zero_u64_kernel(unsigned long long* p, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += stride)
    p[j] = 0ull;
}

__global__ void store_part_kernel(CsPart* out, CsPart v) {
  if (threadIdx.x == 0) *out = v;
}

uint32_t fill_grid(uint64_t n) {
  const uint64_t g = (n + 255) / 256;
  return static_cast<uint32_t>(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

uint32_t checksum_parts(int dt, uint64_t n) {
  const uint64_t p = (n * dtype_size(dt) + kSumChunk * 16 - 1) / (kSumChunk * 16);
  return static_cast<uint32_t>(p < 1 ? 1 : (p > kSumMaxParts ? kSumMaxParts : p));
}

// LDS each first-pass workgroup of the checksum holds (its tree's 8 KiB plus
// an unused dynamic part), which sets how many share a CU's 160 KiB: two for
// binary64 and binary32, three for the 16-bit formats, whose fold spends more
// instructions per byte.  With few resident waves the next chunk's loads
// keep enough bytes in flight.
static uint32_t checksum_dynamic_lds(int dt) {
  constexpr uint32_t kTree = 4 * kReduceBlock * 8;
  return (dt == DT_F64 || dt == DT_F32 ? 64 * 1024 : 48 * 1024) - kTree;
}

// LDS each mismatch-count workgroup holds (its tree's 8 KiB plus an unused
// dynamic part): 64 KiB, two workgroups per CU, as for the binary64 checksum.
static uint32_t mismatch_dynamic_lds() { return 64 * 1024 - 4 * kReduceBlock * 8; }

// The batched fill for storage format dt, constant (U false) or uniform.
#define TS_BY_FORMAT_U(dt, U, ...)                                                             \
  switch (dt) {                                                                                \
    case DT_F64: hipLaunchKernelGGL((batch_fill_kernel<DT_F64, U>), __VA_ARGS__); break;       \
    case DT_F32: hipLaunchKernelGGL((batch_fill_kernel<DT_F32, U>), __VA_ARGS__); break;       \
    case DT_BF16: hipLaunchKernelGGL((batch_fill_kernel<DT_BF16, U>), __VA_ARGS__); break;     \
    case DT_F16: hipLaunchKernelGGL((batch_fill_kernel<DT_F16, U>), __VA_ARGS__); break;       \
    default: return hipErrorInvalidValue;                                                      \
  }                                                                                            \
  return hipGetLastError();

// The checksum's first pass for storage format dt; EM as the kernel's.
#define TS_CHECKSUM_BY_FORMAT(dt, EM, ...)                                                   \
  switch (dt) {                                                                                \
    case DT_F64: hipLaunchKernelGGL((checksum_pass1<DT_F64, EM>), __VA_ARGS__); break;       \
    case DT_F32: hipLaunchKernelGGL((checksum_pass1<DT_F32, EM>), __VA_ARGS__); break;       \
    case DT_BF16: hipLaunchKernelGGL((checksum_pass1<DT_BF16, EM>), __VA_ARGS__); break;     \
    case DT_F16: hipLaunchKernelGGL((checksum_pass1<DT_F16, EM>), __VA_ARGS__); break;       \
    default: return hipErrorInvalidValue;                                                      \
  }

#define TS_BY_FORMAT(dt, KERNEL, ...)                                                          \
  switch (dt) {                                                                                \
    case DT_F64: hipLaunchKernelGGL(KERNEL<DT_F64>, __VA_ARGS__); break;                       \
    case DT_F32: hipLaunchKernelGGL(KERNEL<DT_F32>, __VA_ARGS__); break;                       \
    case DT_BF16: hipLaunchKernelGGL(KERNEL<DT_BF16>, __VA_ARGS__); break;                     \
    case DT_F16: hipLaunchKernelGGL(KERNEL<DT_F16>, __VA_ARGS__); break;                       \
    default: return hipErrorInvalidValue;                                                      \
  }                                                                                            \
  return hipGetLastError();

// Element-wise head up to the first 16-byte boundary, whole 16-byte vectors,
// and the grid for one pass over the vectors: one vector per lane of 256-lane
// workgroups, as many as a launch holds (the kernel strides over any rest).
// A write-only kernel that strides loses speed: the constant fill over 32 GiB
// wrote 5.8 TB/s with a grid capped at 2^20 workgroups and 7.25 TB/s without.
static void vector_split(int dt, const void* p, uint64_t n, uint64_t* head, uint64_t* nvec, uint64_t* grid) {
  const uint64_t es = dtype_size(dt), per = 16 / es;
  const uint64_t a = reinterpret_cast<uintptr_t>(p) % 16;  // a multiple of es
  *head = ((16 - a) % 16) / es;
  if (*head > n) *head = n;
  *nvec = (n - *head) / per;
  const uint64_t g = cap_grid((*nvec + 255) / 256, 256);
  *grid = g < 1 ? 1 : g;
}

// LDS a constant-fill workgroup reserves without using it, so that four share
// a CU: writes alone stream fastest with fewer resident waves.
constexpr uint32_t kFillLds = 40 * 1024;

hipError_t launch_fill_const(int dt, void* p, uint64_t n, double value, hipStream_t s) {
  const uint64_t es = dtype_size(dt);
  const uint64_t a = reinterpret_cast<uintptr_t>(p) % 8;  // a multiple of es
  uint64_t head = ((8 - a) % 8) / es;
  if (head > n) head = n;
  const uint64_t nwords = (n - head) * es / 8;
  uint64_t g = cap_grid((nwords + kFillChunkWords - 1) / kFillChunkWords, 256);  // no stride below 64 GiB
  g = g < 1 ? 1 : g;
  TS_BY_FORMAT(dt, fill_const_kernel, dim3(static_cast<uint32_t>(g)), dim3(256), kFillLds, s, p, n, value, head,
               nwords)
}

hipError_t launch_fill_uniform(int dt, void* p, uint64_t n, uint64_t seed, uint64_t stream_id,
                               uint64_t first_index, double lo, double w, hipStream_t s) {
  const uint64_t state0 = seed ^ (stream_id << 48);
  uint64_t head, nvec, grid;
  vector_split(dt, p, n, &head, &nvec, &grid);
  TS_BY_FORMAT(dt, fill_uniform_kernel, dim3(static_cast<uint32_t>(grid)), dim3(256), 0, s, p, n, state0,
               first_index, lo, w, head, nvec)
}

hipError_t launch_checksum_to(int dt, const void* x, uint64_t n, double expected, CsPart* parts, CsPart* out,
                              hipStream_t s) {
  const uint32_t np = checksum_parts(dt, n);
  const uint32_t lds = checksum_dynamic_lds(dt);
  const dim3 g(np), b(kReduceBlock);
  if (std::isnan(expected)) {
    TS_CHECKSUM_BY_FORMAT(dt, kExpNan, g, b, lds, s, x, n, expected, parts, np)
  } else if (expected == 0.0) {
    TS_CHECKSUM_BY_FORMAT(dt, kExpZero, g, b, lds, s, x, n, expected, parts, np)
  } else {
    TS_CHECKSUM_BY_FORMAT(dt, kExpValue, g, b, lds, s, x, n, expected, parts, np)
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(kReduceBlock), 0, s, parts, np, out);
  return hipGetLastError();
}

hipError_t launch_checksum(int dt, const void* x, uint64_t n, double expected, void* scratch,
                           hipStream_t s) {
  CsPart* parts = static_cast<CsPart*>(scratch);
  return launch_checksum_to(dt, x, n, expected, parts, parts + kReduceMaxParts, s);
}

hipError_t launch_store_part(CsPart* out, const CsPart& v, hipStream_t s) {
  hipLaunchKernelGGL(store_part_kernel, dim3(1), dim3(64), 0, s, out, v);
  return hipGetLastError();
}

hipError_t noalloc_parts(int device, CsPart** out) {
  static std::mutex mu;
  static CsPart* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = static_cast<CsPart*>(p);
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_mismatch(int dt, const void* x, const void* ref, uint64_t n, void* scratch,
                           hipStream_t s) {
  CsPart* parts = static_cast<CsPart*>(scratch);
  const uint32_t np = checksum_parts(dt, n);
  const uint32_t lds = mismatch_dynamic_lds();
  switch (dt) {
    case DT_F64: hipLaunchKernelGGL(mismatch_pass1<DT_F64>, dim3(np), dim3(kReduceBlock), lds, s, x, ref, n, parts, np); break;
    case DT_F32: hipLaunchKernelGGL(mismatch_pass1<DT_F32>, dim3(np), dim3(kReduceBlock), lds, s, x, ref, n, parts, np); break;
    case DT_BF16: hipLaunchKernelGGL(mismatch_pass1<DT_BF16>, dim3(np), dim3(kReduceBlock), lds, s, x, ref, n, parts, np); break;
    case DT_F16: hipLaunchKernelGGL(mismatch_pass1<DT_F16>, dim3(np), dim3(kReduceBlock), lds, s, x, ref, n, parts, np); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(kReduceBlock), 0, s, parts, np, parts + kReduceMaxParts);
  return hipGetLastError();
}

hipError_t launch_batch_fill(int dt, const BatchTile* tiles, uint64_t ntiles, uint32_t per_wg, int which,
                             int uniform, double value, uint64_t seed, uint32_t grid, hipStream_t s) {
  if (per_wg < 1 || per_wg > kAuxMaxTilesPerWg) return hipErrorInvalidValue;
  if (uniform) {
    TS_BY_FORMAT_U(dt, true, dim3(grid), dim3(kAuxBlock), 0, s, tiles, ntiles, per_wg, which, value, seed)
  }
  TS_BY_FORMAT_U(dt, false, dim3(grid), dim3(kAuxBlock), 0, s, tiles, ntiles, per_wg, which, value, seed)
}

hipError_t launch_batch_mismatch(int dt, const BatchTile* tiles, uint64_t ntiles, uint32_t per_wg, int which,
                                 const double* expected, unsigned long long* counts, uint32_t grid,
                                 hipStream_t s) {
  TS_BY_FORMAT(dt, batch_mismatch_kernel, dim3(grid), dim3(kAuxBlock), 0, s, tiles, ntiles, per_wg, which,
               expected, counts)
}

hipError_t launch_zero_u64(unsigned long long* p, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace ts
