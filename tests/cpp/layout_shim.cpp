// layout_shim.cpp -- C entry points over the GPU-free rules of libtstream
// (operand checks, alignment planning, batch tile planning) so the CPU tests
// can exercise them with g++ on a machine without a GPU.
#include <string.h>

#include "ts_layout.hpp"

extern "C" {

int shim_check_map(int uses_y, int exec_dev, const uint64_t* xs, const uint64_t* ys, const uint64_t* ds,
                   uint64_t* count) {
  // each operand: {addr, n, dtype, device}
  ts::Operand x{static_cast<uintptr_t>(xs[0]), xs[1], static_cast<int>(xs[2]), static_cast<int>(xs[3])};
  ts::Operand y{static_cast<uintptr_t>(ys[0]), ys[1], static_cast<int>(ys[2]), static_cast<int>(ys[3])};
  ts::Operand d{static_cast<uintptr_t>(ds[0]), ds[1], static_cast<int>(ds[2]), static_cast<int>(ds[3])};
  ts::MapCheck r = ts::check_map(uses_y != 0, exec_dev, x, &y, d);
  *count = r.count;
  return r.status;
}

int shim_align_class(uint64_t x, int has_y, uint64_t y, uint64_t d) {
  uintptr_t yy = static_cast<uintptr_t>(y);
  return ts::align_class(static_cast<uintptr_t>(x), has_y ? &yy : nullptr, static_cast<uintptr_t>(d));
}

int shim_plan_plain(uint64_t x, int has_y, uint64_t y, uint64_t d, uint64_t count, uint64_t es, uint64_t vb,
                    uint64_t* out) {
  uintptr_t yy = static_cast<uintptr_t>(y);
  ts::PlainPlan p{};
  const bool ok = ts::plan_plain(static_cast<uintptr_t>(x), has_y ? &yy : nullptr, static_cast<uintptr_t>(d),
                                 count, es, vb, p);
  out[0] = p.head;
  out[1] = p.nvec;
  out[2] = p.tail;
  return ok ? 1 : 0;
}

// descs: count x {a, b, c, len}; tiles_out: cap x {inst, start, end};
// meta_out: count x {head, vec_ok}.  Returns the status; *ntiles = tile count.
int shim_plan_batch(const uint64_t* descs, size_t count, uint64_t es, int64_t tile, uint64_t* tiles_out,
                    size_t cap, uint64_t* meta_out, uint64_t* ntiles, uint64_t* total) {
  std::vector<ts::HostDesc> in(count);
  for (size_t i = 0; i < count; ++i)
    in[i] = ts::HostDesc{static_cast<uintptr_t>(descs[4 * i]), static_cast<uintptr_t>(descs[4 * i + 1]),
                         static_cast<uintptr_t>(descs[4 * i + 2]), descs[4 * i + 3], 1.0};
  std::vector<ts::BatchDesc> bd;
  std::vector<ts::BatchTile> bt;
  std::string err;
  uint64_t tot = 0;
  const int st = ts::plan_batch(in.data(), count, es, tile, bd, bt, tot, err);
  if (st != 0) return st;
  *ntiles = bt.size();
  *total = tot;
  for (size_t t = 0; t < bt.size() && t < cap; ++t) {
    tiles_out[3 * t] = bt[t].inst;
    tiles_out[3 * t + 1] = bt[t].start;
    tiles_out[3 * t + 2] = bt[t].start + bt[t].count;
    // every tile carries its instance's pointers, scalar and alignment
    const ts::BatchDesc& d = bd[bt[t].inst];
    if (bt[t].a != d.a || bt[t].b != d.b || bt[t].c != d.c || bt[t].head != d.head ||
        bt[t].vec_ok != d.vec_ok || bt[t].q != d.q)
      return -100;
  }
  for (size_t i = 0; i < count; ++i) {
    meta_out[2 * i] = bd[i].head;
    meta_out[2 * i + 1] = bd[i].vec_ok;
  }
  return 0;
}

// descs: count x {a, b, c, len}; err receives the message (cap bytes).
int shim_check_batch_overlap(const uint64_t* descs, size_t count, uint64_t es, char* err, size_t cap) {
  std::vector<ts::HostDesc> in(count);
  for (size_t i = 0; i < count; ++i)
    in[i] = ts::HostDesc{static_cast<uintptr_t>(descs[4 * i]), static_cast<uintptr_t>(descs[4 * i + 1]),
                         static_cast<uintptr_t>(descs[4 * i + 2]), descs[4 * i + 3], 1.0};
  std::string msg;
  const int st = ts::check_batch_overlap(in.data(), count, es, msg);
  if (cap) {
    strncpy(err, msg.c_str(), cap - 1);
    err[cap - 1] = 0;
  }
  return st;
}

uint64_t shim_cap_grid(uint64_t grid, uint64_t block) { return ts::cap_grid(grid, block); }

}  // extern "C"
