// ts_layout.hpp -- host-side rules of libtstream that need no GPU: operand
// validation for the algorithm calls, alignment planning of a plain launch,
// and the tile planner of batched instances.  Pure C++ (no HIP headers) so
// the rules can be unit-tested on a machine without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace ts {

// Largest grid.x of a launch.
constexpr uint64_t kMaxGridX = 0x7fffffffull;
// The dispatch counts a launch's work-items (grid.x * block) in 32 bits, so
// a launch holds at most 2^32 - 1 of them; a larger one would run only part
// of its grid.
constexpr uint64_t kMaxWorkItems = 0xffffffffull;
// Workgroups of `block` lanes for a grid-stride kernel: `grid`, capped so
// that both limits hold (the kernel's loop covers whatever lies beyond).
inline uint64_t cap_grid(uint64_t grid, uint64_t block) {
  uint64_t cap = kMaxWorkItems / block;
  if (cap > kMaxGridX) cap = kMaxGridX;
  return grid > cap ? cap : grid;
}

// Status codes (same values as ts_status in tstream.h).
enum : int {
  ST_OK = 0,
  ST_INVALID = -1,
  ST_SHAPE = -2,
  ST_DTYPE = -3,
  ST_PLACEMENT = -4,
  ST_ALIAS = -5,
  ST_DEVICE = -6,
  ST_OOM = -7,
  ST_UNSUPPORTED = -8
};

inline size_t dtype_size(int dt) {
  switch (dt) {
    case 0: return 8;
    case 1: return 4;
    case 2:
    case 3: return 2;
    case 4: return 1;
    default: return 0;
  }
}

// One operand of a map as the checks see it.
struct Operand {
  uintptr_t addr;
  uint64_t n;
  int dtype;
  int device;
};

struct MapCheck {
  int status;
  uint64_t count;
  std::string msg;
};

inline bool ranges_overlap(uintptr_t a, uintptr_t b, uint64_t count, size_t es) {
  if (count == 0) return false;
  const uintptr_t bytes = static_cast<uintptr_t>(count) * es;
  return a < b + bytes && b < a + bytes;
}

// Rules of the algorithm calls: count = n of the first input; the other
// operands hold at least count elements; one storage type; every operand on
// the executor's device; dst equal to an input (in place) or disjoint from it.
inline MapCheck check_map(bool uses_y, int exec_device, const Operand& x, const Operand* y,
                          const Operand& d) {
  MapCheck r{ST_OK, x.n, ""};
  const Operand* ops[3] = {&x, uses_y ? y : nullptr, &d};
  const char* names[3] = {"x", "y", "dst"};
  for (int i = 0; i < 3; ++i) {
    if (!ops[i]) continue;
    if (ops[i]->dtype != x.dtype) {
      r.status = ST_DTYPE;
      r.msg = std::string("operand ") + names[i] + " has another storage type than x";
      return r;
    }
  }
  for (int i = 0; i < 3; ++i) {
    if (!ops[i]) continue;
    if (ops[i]->device != exec_device) {
      r.status = ST_PLACEMENT;
      r.msg = std::string("operand ") + names[i] + " is placed on device " +
              std::to_string(ops[i]->device) + ", the executor runs on device " +
              std::to_string(exec_device);
      return r;
    }
  }
  for (int i = 1; i < 3; ++i) {
    if (!ops[i]) continue;
    if (ops[i]->n < x.n) {
      r.status = ST_SHAPE;
      r.msg = std::string("operand ") + names[i] + " holds " + std::to_string(ops[i]->n) +
              " elements, the range needs " + std::to_string(x.n);
      return r;
    }
  }
  const size_t es = dtype_size(x.dtype);
  for (int i = 0; i < 2; ++i) {
    if (!ops[i]) continue;
    if (ops[i]->addr != d.addr && ranges_overlap(ops[i]->addr, d.addr, x.n, es)) {
      r.status = ST_ALIAS;
      r.msg = std::string("dst partly overlaps ") + names[i];
      return r;
    }
  }
  return r;
}

// Alignment class of a map's operands with respect to 16-byte vectors:
// 0 all aligned, 1 one shared misalignment, 2 different misalignments.
inline int align_class(uintptr_t x, const uintptr_t* y, uintptr_t d) {
  const uintptr_t m = d % 16;
  if (x % 16 != m || (y && *y % 16 != m)) return 2;
  return m == 0 ? 0 : 1;
}

// Split [0, count) of a plain launch into an element-wise head, a body of
// whole vb-byte vectors and an element-wise tail.  When every operand has the
// same misalignment modulo a 128-byte cache line, the head runs up to a line
// boundary, so each wave's 1 KiB accesses cover whole lines; otherwise only
// up to a vb boundary.  Returns false when the misalignments differ modulo
// vb, in which case only vb == element size can be used.
struct PlainPlan {
  uint64_t head, nvec, tail;
};

constexpr uintptr_t kLineBytes = 128;

inline bool plan_plain(uintptr_t x, const uintptr_t* y, uintptr_t d, uint64_t count, size_t es,
                       size_t vb, PlainPlan& out) {
  const uintptr_t m = d % vb;
  if (x % vb != m || (y && *y % vb != m)) return false;
  const uintptr_t ml = d % kLineBytes;
  const bool line = x % kLineBytes == ml && (!y || *y % kLineBytes == ml);
  const uintptr_t unit = line ? kLineBytes : vb;
  const uintptr_t mu = d % unit;
  const uint64_t v = vb / es;
  uint64_t head = mu == 0 ? 0 : (unit - mu) / es;
  if (head > count) head = count;
  const uint64_t rest = count - head;
  out.head = head;
  out.nvec = rest / v;
  out.tail = rest % v;
  return true;
}

// ---------------------------------------------------------------------------
// Batched instances.
// ---------------------------------------------------------------------------

// Device descriptor of one instance.  `head` = elements before the first
// 16-byte aligned element (the same for a, b and c when vec_ok is set).
struct BatchDesc {
  const void* a;
  const void* b;
  const void* c;
  uint64_t len;
  double q;
  float qf;
  uint32_t head;
  uint32_t vec_ok;
  uint32_t pad;
};

// One tile: the element range [start, start + count) of one instance, with
// everything a workgroup needs to stream it (64 bytes, one scalar load).
// Boundaries other than 0 and len sit at head + k * tile_elems, so only an
// instance's first tile has an unaligned head and only its last tile a
// ragged tail.
struct BatchTile {
  const void* a;
  const void* b;
  const void* c;
  uint64_t start;
  uint64_t count;
  double q;
  float qf;
  uint32_t head;    // the instance's head (elements before 16-byte alignment)
  uint32_t inst;
  uint32_t vec_ok;  // a, b and c share one misalignment
};
static_assert(sizeof(BatchTile) == 64, "tile records are one 64-byte scalar load");

struct HostDesc {
  uintptr_t a, b, c;
  uint64_t len;
  double q;
};

// Overlap rule of a batch (one launch runs every instance at once, so
// instances that share memory would race): inside one instance a, b and c
// are each either the very same array or disjoint from one another (in
// place, as the algorithm calls allow); arrays of different instances never
// share a byte.  Instances of length 0 hold no memory.  Returns ST_OK,
// ST_SHAPE when a range runs past the end of the address space, or ST_ALIAS
// naming the first overlapping pair.
inline int check_batch_overlap(const HostDesc* in, size_t count, size_t es, std::string& err) {
  struct Range {
    uintptr_t lo, hi;
    size_t inst;
    int which;
  };
  static const char* const kNames[3] = {"a", "b", "c"};
  std::vector<Range> r;
  r.reserve(3 * count);
  for (size_t i = 0; i < count; ++i) {
    const HostDesc& h = in[i];
    if (h.len == 0) continue;
    const uintptr_t p[3] = {h.a, h.b, h.c};
    for (int w = 0; w < 3; ++w) {
      bool same = false;  // the same array as an earlier one of this instance
      for (int v = 0; v < w; ++v) same = same || p[v] == p[w];
      if (same) continue;
      if (es == 0 || h.len > (UINTPTR_MAX - p[w]) / es) {
        err = "instance " + std::to_string(i) + ": array " + kNames[w] + " runs past the end of the address space";
        return ST_SHAPE;
      }
      r.push_back(Range{p[w], p[w] + static_cast<uintptr_t>(h.len * es), i, w});
    }
  }
  std::sort(r.begin(), r.end(), [](const Range& x, const Range& y) {
    return x.lo != y.lo ? x.lo < y.lo : x.hi < y.hi;
  });
  size_t reach = 0;  // the range reaching furthest so far
  for (size_t k = 1; k < r.size(); ++k) {
    if (r[k].lo < r[reach].hi) {
      const Range& x = r[reach];
      const Range& y = r[k];
      if (x.inst == y.inst)
        err = "instance " + std::to_string(x.inst) + ": arrays " + kNames[x.which] + " and " + kNames[y.which] +
              " partly overlap";
      else
        err = "instances " + std::to_string(std::min(x.inst, y.inst)) + " and " +
              std::to_string(std::max(x.inst, y.inst)) + " share memory (arrays " + kNames[x.which] + " and " +
              kNames[y.which] + ")";
      return ST_ALIAS;
    }
    if (r[k].hi > r[reach].hi) reach = k;
  }
  return ST_OK;
}

// Build the device descriptors and the tile table.  Tiles of one instance
// are consecutive in the table; instances follow one another in order.
inline int plan_batch(const HostDesc* in, size_t count, size_t es, int64_t tile_elems,
                      std::vector<BatchDesc>& descs, std::vector<BatchTile>& tiles,
                      uint64_t& total, std::string& err) {
  if (es == 0) {
    err = "unknown storage type";
    return ST_INVALID;
  }
  if (tile_elems <= 0 || tile_elems % 8 != 0) {
    err = "tile_elems must be a positive multiple of 8";
    return ST_INVALID;
  }
  if (count > 0xffffffffull) {
    err = "too many instances";
    return ST_INVALID;
  }
  descs.assign(count, BatchDesc{});
  tiles.clear();
  total = 0;
  const uint64_t T = static_cast<uint64_t>(tile_elems);
  for (size_t i = 0; i < count; ++i) {
    const HostDesc& h = in[i];
    if (h.len > 0 && (!h.a || !h.b || !h.c)) {
      err = "instance " + std::to_string(i) + ": NULL array with len > 0";
      return ST_INVALID;
    }
    if (h.a % es || h.b % es || h.c % es) {
      err = "instance " + std::to_string(i) + ": array not aligned to its element size";
      return ST_INVALID;
    }
    BatchDesc& d = descs[i];
    d.a = reinterpret_cast<const void*>(h.a);
    d.b = reinterpret_cast<const void*>(h.b);
    d.c = reinterpret_cast<const void*>(h.c);
    d.len = h.len;
    d.q = h.q;
    d.qf = static_cast<float>(h.q);
    const uintptr_t m = h.c % 16;
    d.vec_ok = (h.a % 16 == m && h.b % 16 == m) ? 1u : 0u;
    d.head = d.vec_ok && m ? static_cast<uint32_t>((16 - m) / es) : 0u;
    total += h.len;
    if (h.len == 0) continue;
    const uint64_t hd = d.head < h.len ? d.head : h.len;
    uint64_t start = 0;
    uint64_t end = hd + T < h.len ? hd + T : h.len;
    for (;;) {
      tiles.push_back(BatchTile{d.a, d.b, d.c, start, end - start, d.q, d.qf, d.head,
                                static_cast<uint32_t>(i), d.vec_ok});
      if (end >= h.len) break;
      start = end;
      end = end + T < h.len ? end + T : h.len;
    }
  }
  return ST_OK;
}

}  // namespace ts
