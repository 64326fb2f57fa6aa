// tune.hpp -- the launch-configuration table of libtstream.
//
// Key: (op, storage type, size bucket floor(log2 n), alignment class,
// batched).  Lookup order: a forced configuration for (op, type, batched);
// the exact key; the nearest size bucket with the same other fields; the
// built-in default.  Pure C++ (no HIP): the table and its JSON form can be
// exercised without a GPU.
#pragma once

#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tstream.h"

namespace ts {

struct TuneKey {
  int op, dtype, bucket, align, batched;
  bool operator<(const TuneKey& o) const {
    return std::tie(op, dtype, bucket, align, batched) <
           std::tie(o.op, o.dtype, o.bucket, o.align, o.batched);
  }
};

struct TuneEntry {
  ts_kernel_cfg cfg;
  double bytes_per_s;
};

int size_bucket(uint64_t n);
ts_kernel_cfg default_cfg(int batched, int dtype);
// Empty string if cfg is a valid configuration (plain or batched), else why not.
std::string cfg_problem(const ts_kernel_cfg& cfg, int batched);
std::vector<ts_kernel_cfg> candidates(int batched);

class TuneTable {
 public:
  ts_kernel_cfg lookup(int op, int dtype, uint64_t n, int align, int batched) const;
  void put(const TuneKey& k, const TuneEntry& e);
  void force(int op, int dtype, int batched, const ts_kernel_cfg* cfg);
  void clear();
  // Returns 0, or a negative status with *err set (table unchanged on error).
  int load(const std::string& path, std::string* err);
  int save(const std::string& path, std::string* err) const;
  std::string to_json() const;
  int from_json(const std::string& text, std::string* err);

 private:
  mutable std::mutex mu_;
  std::map<TuneKey, TuneEntry> entries_;
  bool forced_set_[4][4][2] = {};
  ts_kernel_cfg forced_[4][4][2] = {};
};

TuneTable& tune_table();

}  // namespace ts
