// ts_device.hpp -- gfx950 device code for the STREAM maps (Section 5,
// Listing 4 of Heller et al.): copy, scale, add, triad over placed arrays.
//
// Design (CDNA4, HBM-bound, no matrix cores: nothing here is a contraction):
//  * every lane moves VB bytes per access (16 B -> global_load/store_dwordx4),
//    so one wave instruction covers 1 KiB of contiguous memory;
//  * U independent vectors per lane are loaded before any is stored, giving
//    U (or 2U) loads in flight per lane without LDS or barriers;
//  * optional nontemporal hints on loads and stores (streaming data is never
//    reused);
//  * either one pass (grid covers the array once) or a grid-stride loop over
//    a fixed grid; both keep element ownership disjoint, so results do not
//    depend on the launch shape;
//  * reduced-precision storage widens exactly to binary32, evaluates the map
//    in binary32 and rounds back to nearest-even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ts_internal.hpp"

namespace ts {

enum : int { OP_COPY = 0, OP_SCALE = 1, OP_ADD = 2, OP_TRIAD = 3 };
enum : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3 };

// Storage type T and arithmetic type C of each storage format.
template <int DT> struct Fmt;
template <> struct Fmt<DT_F64> { using T = double; using C = double; };
template <> struct Fmt<DT_F32> { using T = float; using C = float; };
template <> struct Fmt<DT_BF16> { using T = uint16_t; using C = float; };
template <> struct Fmt<DT_F16> { using T = uint16_t; using C = float; };

// Keep a binary32 result in a register as it is, so the compiler cannot fold
// the multiply or add into a mixed-precision instruction that rounds once,
// straight to 16 bits: the map is defined as binary32 arithmetic followed by
// a separate rounding to the storage format.
__device__ __forceinline__ float materialize(float v) {
  asm("" : "+v"(v));
  return v;
}

template <int DT>
__device__ __forceinline__ typename Fmt<DT>::C widen(typename Fmt<DT>::T v) {
  if constexpr (DT == DT_BF16) {
    return __builtin_bit_cast(float, static_cast<uint32_t>(v) << 16);
  } else if constexpr (DT == DT_F16) {
    return static_cast<float>(__builtin_bit_cast(_Float16, v));
  } else {
    return v;
  }
}

// Round-to-nearest-even narrowing (the hardware conversions use the MODE
// register's rounding, which is nearest-even).
template <int DT>
__device__ __forceinline__ typename Fmt<DT>::T narrow(typename Fmt<DT>::C v) {
  if constexpr (DT == DT_BF16) {
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(materialize(v)));
  } else if constexpr (DT == DT_F16) {
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(materialize(v)));
  } else {
    return v;
  }
}

template <int OP, typename C>
__device__ __forceinline__ C apply(C x, C y, C q) {
  if constexpr (OP == OP_SCALE) {
    return q * x;
  } else if constexpr (OP == OP_ADD) {
    return x + y;
  } else if constexpr (OP == OP_TRIAD) {
    if constexpr (sizeof(C) == 8) return __builtin_fma(q, y, x);
    else return __builtin_fmaf(q, y, x);
  } else {
    return x;
  }
}

template <int OP> constexpr bool uses_y() { return OP == OP_ADD || OP == OP_TRIAD; }

// Raw lane vector of VB bytes.
template <int VB> struct Raw;
template <> struct Raw<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };
template <> struct Raw<8> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <> struct Raw<4> { typedef uint32_t type; };
template <> struct Raw<2> { typedef uint16_t type; };

// Every operand of these kernels is device (global) memory.  Accesses go
// through global-address-space pointers, so they compile to global_load /
// global_store even when the pointer was read from memory (a batch's tile
// records) rather than passed as a kernel argument: the flat forms the
// compiler would otherwise emit also count against the scalar-memory wait
// counter, which ties every store to outstanding scalar loads.
template <class T> using Global = __attribute__((address_space(1))) T;

template <class T>
__device__ __forceinline__ const Global<T>* global_ptr(const T* p) {
  return (const Global<T>*)p;
}

template <class T>
__device__ __forceinline__ Global<T>* global_ptr(T* p) {
  return (Global<T>*)p;
}

template <int VB, bool NT>
__device__ __forceinline__ typename Raw<VB>::type load(const void* p) {
  using R = typename Raw<VB>::type;
  const Global<R>* g = global_ptr(static_cast<const R*>(p));
  if constexpr (NT) return __builtin_nontemporal_load(g);
  else return *g;
}

template <int VB, bool NT>
__device__ __forceinline__ void store(void* p, typename Raw<VB>::type v) {
  using R = typename Raw<VB>::type;
  Global<R>* g = global_ptr(static_cast<R*>(p));
  if constexpr (NT) __builtin_nontemporal_store(v, g);
  else *g = v;
}

template <typename T, int VB> union Pack {
  typename Raw<VB>::type raw;
  T e[VB / sizeof(T)];
};

// The map over one raw vector.  Copy moves the bits unchanged.
template <int DT, int OP, int VB>
__device__ __forceinline__ typename Raw<VB>::type map_vec(typename Raw<VB>::type rx,
                                                          typename Raw<VB>::type ry,
                                                          typename Fmt<DT>::C q) {
  if constexpr (OP == OP_COPY) {
    return rx;
  } else {
    using T = typename Fmt<DT>::T;
    constexpr int V = VB / sizeof(T);
    Pack<T, VB> px, py, pd;
    px.raw = rx;
    py.raw = ry;
#pragma unroll
    for (int k = 0; k < V; ++k)
      pd.e[k] = narrow<DT>(apply<OP>(widen<DT>(px.e[k]), widen<DT>(py.e[k]), q));
    return pd.raw;
  }
}

// The map on element j (head, tail and element-wise paths).
template <int DT, int OP>
__device__ __forceinline__ void map_elem(const typename Fmt<DT>::T* x, const typename Fmt<DT>::T* y,
                                         typename Fmt<DT>::T* d, typename Fmt<DT>::C q, uint64_t j) {
  if constexpr (OP == OP_COPY) {
    global_ptr(d)[j] = global_ptr(x)[j];
  } else {
    typename Fmt<DT>::C yv = 0;
    if constexpr (uses_y<OP>()) yv = widen<DT>(global_ptr(y)[j]);
    global_ptr(d)[j] = narrow<DT>(apply<OP>(widen<DT>(global_ptr(x)[j]), yv, q));
  }
}

template <int DT>
__device__ __forceinline__ typename Fmt<DT>::C pick_q(double q, float qf) {
  if constexpr (sizeof(typename Fmt<DT>::C) == 8) return q;
  else return qf;
}

// Vector body over nvec VB-byte vectors starting at xb/yb/db (all VB-aligned):
// lane `lane` of a group of `width` lanes handles vectors v0, v0+width, ...
// U at a time, starting at `first`, with stride `step` between groups.
template <int DT, int OP, int VB, int U, bool NTL, bool NTS>
__device__ __forceinline__ void vec_body(const char* xb, const char* yb, char* db,
                                         typename Fmt<DT>::C q, uint64_t nvec, uint64_t first,
                                         uint64_t width, uint64_t step) {
  using R = typename Raw<VB>::type;
  for (uint64_t v0 = first; v0 < nvec; v0 += step) {
    if (v0 + (U - 1) * width < nvec) {
      R rx[U], ry[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        rx[k] = load<VB, NTL>(xb + (v0 + k * width) * VB);
        if constexpr (uses_y<OP>()) ry[k] = load<VB, NTL>(yb + (v0 + k * width) * VB);
        else ry[k] = rx[k];
      }
#pragma unroll
      for (int k = 0; k < U; ++k)
        store<VB, NTS>(db + (v0 + k * width) * VB, map_vec<DT, OP, VB>(rx[k], ry[k], q));
    } else {
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const uint64_t v = v0 + k * width;
        if (v < nvec) {
          R rx = load<VB, NTL>(xb + v * VB);
          R ry = rx;
          if constexpr (uses_y<OP>()) ry = load<VB, NTL>(yb + v * VB);
          store<VB, NTS>(db + v * VB, map_vec<DT, OP, VB>(rx, ry, q));
        }
      }
    }
  }
}

// Plain kernel: elements [0, head) and the `tail` elements after the vector
// body are done one per lane by the first lanes of the grid; the body covers
// nvec vectors of VB bytes starting at element `head`.
template <int DT, int OP, int VB, int U, bool NTL, bool NTS>
__global__ __launch_bounds__(1024) void stream_kernel(const void* xv, const void* yv, void* dv,
                                                      double q, float qf, uint64_t head,
                                                      uint64_t nvec, uint64_t tail) {
  using T = typename Fmt<DT>::T;
  constexpr int V = VB / sizeof(T);
  const T* x = static_cast<const T*>(xv);
  const T* y = static_cast<const T*>(yv);
  T* d = static_cast<T*>(dv);
  const typename Fmt<DT>::C qc = pick_q<DT>(q, qf);
  const uint64_t width = blockDim.x;
  const uint64_t gid = static_cast<uint64_t>(blockIdx.x) * width + threadIdx.x;
  if (gid < head) map_elem<DT, OP>(x, y, d, qc, gid);
  if (gid < tail) map_elem<DT, OP>(x, y, d, qc, head + nvec * V + gid);
  const char* xb = reinterpret_cast<const char*>(x + head);
  const char* yb = reinterpret_cast<const char*>(y + head);
  char* db = reinterpret_cast<char*>(d + head);
  vec_body<DT, OP, VB, U, NTL, NTS>(xb, yb, db, qc, nvec,
                                    static_cast<uint64_t>(blockIdx.x) * width * U + threadIdx.x,
                                    width, static_cast<uint64_t>(gridDim.x) * width * U);
}

// ---------------------------------------------------------------------------
// Batched ragged instances.
// ---------------------------------------------------------------------------

template <int OP>
__device__ __forceinline__ void roles(const BatchTile& tl, const void*& x, const void*& y, void*& d) {
  // Listing 4 roles inside every instance.
  if constexpr (OP == OP_COPY) { x = tl.a; y = nullptr; d = const_cast<void*>(tl.c); }
  else if constexpr (OP == OP_SCALE) { x = tl.c; y = nullptr; d = const_cast<void*>(tl.b); }
  else if constexpr (OP == OP_ADD) { x = tl.a; y = tl.b; d = const_cast<void*>(tl.c); }
  else { x = tl.b; y = tl.c; d = const_cast<void*>(tl.a); }
}

// The part of one tile a workgroup streams: element-wise ranges [start, vs)
// and [ve, end) around the 16-byte vectors [vs, ve) (only the first tile of
// an instance has a head, only its last a ragged tail).
template <int DT>
struct TileSpan {
  const typename Fmt<DT>::T* x;
  const typename Fmt<DT>::T* y;
  typename Fmt<DT>::T* d;
  typename Fmt<DT>::C q;
  uint64_t start, vs, ve, end;
};

template <int DT, int OP>
__device__ __forceinline__ TileSpan<DT> tile_span(const BatchTile& tl) {
  using T = typename Fmt<DT>::T;
  constexpr uint64_t V = 16 / sizeof(T);
  const void *xv, *yv;
  void* dv;
  roles<OP>(tl, xv, yv, dv);
  TileSpan<DT> s;
  s.x = static_cast<const T*>(xv);
  s.y = static_cast<const T*>(yv);
  s.d = static_cast<T*>(dv);
  s.q = pick_q<DT>(tl.q, tl.qf);
  s.start = tl.start;
  s.end = tl.start + tl.count;
  // The vector middle is computed whether or not the instance has one, and
  // then chosen; the empty asm takes both fields up front, so the record
  // arrives in one round of scalar loads instead of a second one for the
  // field the compiler would otherwise fetch late.
  const uint32_t ok = tl.vec_ok;
  const uint64_t h = tl.head;
  asm volatile("" ::"s"(ok), "s"(tl.head));
  uint64_t vs = s.start < h ? h : h + (s.start - h + V - 1) / V * V;
  if (vs > s.end) vs = s.end;
  uint64_t ve = s.end < h ? vs : h + (s.end - h) / V * V;
  if (ve < vs) ve = vs;
  s.vs = ok ? vs : s.end;
  s.ve = ok ? ve : s.end;
  return s;
}

template <int DT, int OP>
__device__ __forceinline__ void tile_edges(const TileSpan<DT>& s, uint64_t lane, uint64_t width) {
  for (uint64_t j = s.start + lane; j < s.vs; j += width) map_elem<DT, OP>(s.x, s.y, s.d, s.q, j);
  for (uint64_t j = s.ve + lane; j < s.end; j += width) map_elem<DT, OP>(s.x, s.y, s.d, s.q, j);
}

// Tiles between a workgroup and the one whose record it reads ahead (one
// workgroup per tile): a multiple of the 8 XCDs, about one round of the
// workgroups resident on an XCD (32 CUs x 8 workgroups of 256 lanes).
constexpr uint64_t kRecordAhead = 2048;

// One launch over every instance.
//
// K = 1: workgroup w takes tiles w, w + G, w + 2G, ... (G = grid size).
// With one workgroup per tile (G = number of tiles) each workgroup takes one
// tile, and with AHEAD it also reads a record further on (below); with a
// smaller grid the workgroups persist and stride, fetching the next tile
// record while the current tile streams.
//
// K > 1: workgroup w takes the K consecutive tiles Kw .. Kw + K - 1 (then
// Kw + KG, ... on a persistent grid).  It reads the K records together and
// issues the first U vectors per lane of every one of its tiles before it
// stores any, so K*U loads (or 2*K*U) are in flight per lane and one record
// latency serves K tiles; the tiles may belong to different instances.
// Vectors beyond the first U*width of a tile, and the element-wise head and
// tail, follow.
//
// Inside a tile the lanes stream 16-byte vectors like the plain kernel, and
// element ownership is disjoint, so results do not depend on K, U or G.
template <int DT, int OP, int U, int K, bool NTL, bool NTS, bool AHEAD>
__global__ __launch_bounds__(1024) void batch_kernel(const BatchTile* __restrict__ tiles,
                                                     uint64_t ntiles) {
  using T = typename Fmt<DT>::T;
  constexpr int VB = 16;
  constexpr uint64_t V = VB / sizeof(T);
  const uint64_t width = blockDim.x;
  const uint64_t lane = threadIdx.x;
  if constexpr (K == 1) {
    uint64_t t = blockIdx.x;
    if (t >= ntiles) return;
    BatchTile cur = tiles[t];
    uint64_t ahead = 0;
    for (; t < ntiles; t += gridDim.x) {
      BatchTile nxt = cur;
      if (t + gridDim.x < ntiles) nxt = tiles[t + gridDim.x];
      const TileSpan<DT> s = tile_span<DT, OP>(cur);
      // AHEAD (one workgroup per tile): read the record of the tile that a
      // workgroup kRecordAhead later takes.  Workgroups are handed to the
      // XCDs in turn and kRecordAhead is a multiple of their count, so the
      // record lands in the L2 of the XCD that will run that workgroup,
      // which then finds it there instead of waiting on memory before its
      // first data load.  The read depends on this tile's record (a tile is
      // never empty), so it is issued after that record has arrived, and is
      // waited for only at the end: it costs this workgroup no latency.
      if constexpr (AHEAD) {
        if (gridDim.x >= ntiles && s.end > s.start && t + kRecordAhead < ntiles) ahead = tiles[t + kRecordAhead].count;
      }
      const uint64_t nvec = (s.ve - s.vs) / V;
      if (nvec) {
        vec_body<DT, OP, VB, U, NTL, NTS>(reinterpret_cast<const char*>(s.x + s.vs),
                                          reinterpret_cast<const char*>(s.y + s.vs),
                                          reinterpret_cast<char*>(s.d + s.vs), s.q, nvec, lane, width,
                                          width * U);
      }
      tile_edges<DT, OP>(s, lane, width);
      cur = nxt;
    }
    asm volatile("" ::"s"(ahead));  // the read above completes before the workgroup ends
  } else {
    using R = typename Raw<VB>::type;
    for (uint64_t t0 = static_cast<uint64_t>(blockIdx.x) * K; t0 < ntiles;
         t0 += static_cast<uint64_t>(gridDim.x) * K) {
      TileSpan<DT> s[K];
      uint64_t nvec[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        nvec[k] = 0;
        if (t0 + k < ntiles) {
          s[k] = tile_span<DT, OP>(tiles[t0 + k]);
          nvec[k] = (s[k].ve - s[k].vs) / V;
        }
      }
      R rx[K][U], ry[K][U];
#pragma unroll
      for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t v = lane + u * width;
          if (v < nvec[k]) {
            rx[k][u] = load<VB, NTL>(s[k].x + s[k].vs + v * V);
            if constexpr (uses_y<OP>()) ry[k][u] = load<VB, NTL>(s[k].y + s[k].vs + v * V);
            else ry[k][u] = rx[k][u];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t v = lane + u * width;
          if (v < nvec[k])
            store<VB, NTS>(s[k].d + s[k].vs + v * V, map_vec<DT, OP, VB>(rx[k][u], ry[k][u], s[k].q));
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (nvec[k] > U * width) {
          vec_body<DT, OP, VB, U, NTL, NTS>(reinterpret_cast<const char*>(s[k].x + s[k].vs),
                                            reinterpret_cast<const char*>(s[k].y + s[k].vs),
                                            reinterpret_cast<char*>(s[k].d + s[k].vs), s[k].q, nvec[k],
                                            U * width + lane, width, width * U);
        }
        if (t0 + k < ntiles) tile_edges<DT, OP>(s[k], lane, width);
      }
    }
  }
}

// Pieces: 2^PL one-wave workgroups share each tile.  Workgroup w takes
// piece p = w mod P of tile t = w / P: vector p*64 + lane of the tile's
// aligned middle, then every (P*64)-th after it; piece 0 also takes the
// element-wise head and tail.  Consecutive workgroups go to different CUs,
// so a tile's pieces stream from many CUs at once, as the plain kernel's
// one-wave shape does, and the P workgroups of a tile read its record from
// one cache line.  The grid strides over whatever lies beyond it; the host
// launches at least one and at most ntiles * P workgroups, so every
// workgroup has a first piece (the loop tests only before the next one, and
// the first record load waits on nothing but the kernel arguments).
template <int DT, int OP, int VB, bool NTL, bool NTS>
__global__ __launch_bounds__(64) void batch_piece_kernel(const BatchTile* __restrict__ tiles, uint64_t ntiles,
                                                         uint32_t pieces_log2) {
  using T = typename Fmt<DT>::T;
  using R = typename Raw<VB>::type;
  constexpr uint64_t V = VB / sizeof(T);
  const uint64_t P = 1ull << pieces_log2;
  const uint64_t lane = threadIdx.x;
  const uint64_t total = ntiles << pieces_log2;
  uint64_t w = blockIdx.x;
  do {
    const uint64_t t = w >> pieces_log2, p = w & (P - 1);
    const TileSpan<DT> s = tile_span<DT, OP>(tiles[t]);
    const uint64_t nvec = (s.ve - s.vs) / V;
    for (uint64_t v = p * 64 + lane; v < nvec; v += P * 64) {
      const R rx = load<VB, NTL>(s.x + s.vs + v * V);
      R ry;
      if constexpr (uses_y<OP>()) ry = load<VB, NTL>(s.y + s.vs + v * V);
      else ry = rx;
      store<VB, NTS>(s.d + s.vs + v * V, map_vec<DT, OP, VB>(rx, ry, s.q));
    }
    if (p == 0) tile_edges<DT, OP>(s, lane, 64);
    w += gridDim.x;
  } while (w < total);
}

template <int DT, int OP, int VB, int U, bool NTL, bool NTS>
hipError_t launch_plain_inst(const PlainLaunch& L) {
  hipLaunchKernelGGL((stream_kernel<DT, OP, VB, U, NTL, NTS>), dim3(L.grid), dim3(L.block), 0,
                     L.stream, L.x, L.y, L.d, L.q, L.qf, L.head, L.nvec, L.tail);
  return hipGetLastError();
}

template <int DT, int OP, int VB, int U>
hipError_t plain_nt(const PlainLaunch& L) {
  if (L.ntl) {
    return L.nts ? launch_plain_inst<DT, OP, VB, U, true, true>(L)
                 : launch_plain_inst<DT, OP, VB, U, true, false>(L);
  }
  return L.nts ? launch_plain_inst<DT, OP, VB, U, false, true>(L)
               : launch_plain_inst<DT, OP, VB, U, false, false>(L);
}

template <int DT, int OP, int VB>
hipError_t plain_u(const PlainLaunch& L) {
  switch (L.unroll) {
    case 1: return plain_nt<DT, OP, VB, 1>(L);
    case 2: return plain_nt<DT, OP, VB, 2>(L);
    case 4: return plain_nt<DT, OP, VB, 4>(L);
    case 8: return plain_nt<DT, OP, VB, 8>(L);
    default: return hipErrorInvalidValue;
  }
}

template <int DT, int OP>
hipError_t plain_vb(const PlainLaunch& L) {
  constexpr int ES = sizeof(typename Fmt<DT>::T);
  switch (L.vb) {
    case 16: return plain_u<DT, OP, 16>(L);
    case 8: return plain_u<DT, OP, 8>(L);
    default:
      if (L.vb == ES) return plain_u<DT, OP, ES>(L);
      return hipErrorInvalidValue;
  }
}

template <int DT>
hipError_t plain_dispatch(const PlainLaunch& L) {
  switch (L.op) {
    case OP_COPY: return plain_vb<DT, OP_COPY>(L);
    case OP_SCALE: return plain_vb<DT, OP_SCALE>(L);
    case OP_ADD: return plain_vb<DT, OP_ADD>(L);
    case OP_TRIAD: return plain_vb<DT, OP_TRIAD>(L);
    default: return hipErrorInvalidValue;
  }
}

template <int DT, int OP, int U, int K, bool NTL, bool NTS>
hipError_t launch_batch_inst(const BatchLaunch& L) {
  if constexpr (K == 1) {
    if (L.record_ahead) {
      hipLaunchKernelGGL((batch_kernel<DT, OP, U, K, NTL, NTS, true>), dim3(L.grid), dim3(L.block), 0, L.stream,
                         L.tiles, L.ntiles);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((batch_kernel<DT, OP, U, K, NTL, NTS, false>), dim3(L.grid), dim3(L.block), 0, L.stream,
                     L.tiles, L.ntiles);
  return hipGetLastError();
}

template <int DT, int OP, int U, int K>
hipError_t batch_nt(const BatchLaunch& L) {
  if (L.ntl) {
    return L.nts ? launch_batch_inst<DT, OP, U, K, true, true>(L)
                 : launch_batch_inst<DT, OP, U, K, true, false>(L);
  }
  return L.nts ? launch_batch_inst<DT, OP, U, K, false, true>(L)
               : launch_batch_inst<DT, OP, U, K, false, false>(L);
}

// Several tiles per workgroup come with at most two vectors per lane each
// (the candidate set and the configuration check hold to this).
template <int DT, int OP, int U>
hipError_t batch_k(const BatchLaunch& L) {
  if constexpr (U <= 2) {
    switch (L.tiles_per_wg) {
      case 2: return batch_nt<DT, OP, U, 2>(L);
      case 4: return batch_nt<DT, OP, U, 4>(L);
      case 8: return batch_nt<DT, OP, U, 8>(L);
      default: break;
    }
  }
  if (L.tiles_per_wg != 1) return hipErrorInvalidValue;
  return batch_nt<DT, OP, U, 1>(L);
}

template <int DT, int OP>
hipError_t batch_u(const BatchLaunch& L) {
  switch (L.unroll) {
    case 1: return batch_k<DT, OP, 1>(L);
    case 2: return batch_k<DT, OP, 2>(L);
    case 4: return batch_k<DT, OP, 4>(L);
    case 8: return batch_k<DT, OP, 8>(L);
    default: return hipErrorInvalidValue;
  }
}

template <int DT, int OP, int VB, bool NTL, bool NTS>
hipError_t launch_piece_inst(const BatchLaunch& L) {
  hipLaunchKernelGGL((batch_piece_kernel<DT, OP, VB, NTL, NTS>), dim3(L.grid), dim3(64), 0, L.stream, L.tiles,
                     L.ntiles, static_cast<uint32_t>(L.pieces_log2));
  return hipGetLastError();
}

template <int DT, int OP, int VB>
hipError_t piece_nt(const BatchLaunch& L) {
  if (L.ntl) {
    return L.nts ? launch_piece_inst<DT, OP, VB, true, true>(L) : launch_piece_inst<DT, OP, VB, true, false>(L);
  }
  return L.nts ? launch_piece_inst<DT, OP, VB, false, true>(L) : launch_piece_inst<DT, OP, VB, false, false>(L);
}

template <int DT, int OP>
hipError_t batch_pieces(const BatchLaunch& L) {
  if (L.block != 64) return hipErrorInvalidValue;
  switch (L.vb) {
    case 16: return piece_nt<DT, OP, 16>(L);
    case 8: return piece_nt<DT, OP, 8>(L);
    default: return hipErrorInvalidValue;
  }
}

template <int DT>
hipError_t batch_dispatch(const BatchLaunch& L) {
  if (L.pieces_log2 > 0) {
    switch (L.op) {
      case OP_COPY: return batch_pieces<DT, OP_COPY>(L);
      case OP_SCALE: return batch_pieces<DT, OP_SCALE>(L);
      case OP_ADD: return batch_pieces<DT, OP_ADD>(L);
      case OP_TRIAD: return batch_pieces<DT, OP_TRIAD>(L);
      default: return hipErrorInvalidValue;
    }
  }
  switch (L.op) {
    case OP_COPY: return batch_u<DT, OP_COPY>(L);
    case OP_SCALE: return batch_u<DT, OP_SCALE>(L);
    case OP_ADD: return batch_u<DT, OP_ADD>(L);
    case OP_TRIAD: return batch_u<DT, OP_TRIAD>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ts
