// tune.cpp -- launch-configuration table, candidate sets and JSON persistence.
#include "tune.hpp"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace ts {

namespace {
const char* kOpNames[4] = {"copy", "scale", "add", "triad"};
const char* kTypeNames[4] = {"f64", "f32", "bf16", "f16"};
constexpr int kFormatVersion = 1;

int index_of(const char* const* names, int count, const std::string& s) {
  for (int i = 0; i < count; ++i)
    if (s == names[i]) return i;
  return -1;
}
}  // namespace

int size_bucket(uint64_t n) {
  int b = 0;
  while (n > 1) {
    n >>= 1;
    ++b;
  }
  return b;
}

ts_kernel_cfg default_cfg(int batched, int dtype) {
  ts_kernel_cfg c{};
  c.vec_bytes = 16;
  c.nt_store = 1;
  if (batched) {
    // One workgroup of 256 lanes per tile, one 16-byte vector per lane: tiles
    // of 4 KiB per array, the shape the tuner picks for binary64 on the
    // ragged batch.
    const int64_t es = dtype == TS_F64 ? 8 : dtype == TS_F32 ? 4 : 2;
    c.block = 256;
    c.unroll = 1;
    c.nt_load = 1;
    c.grid_per_cu = 0;
    c.tile_elems = 4096 / es;
    c.tiles_per_wg = 1;
    c.wgs_per_tile = 1;
  } else {
    c.block = 256;
    c.unroll = 4;
    c.nt_load = 0;
    c.grid_per_cu = 0;
    c.tile_elems = 0;
    c.tiles_per_wg = 1;
    c.wgs_per_tile = 1;
  }
  return c;
}

std::string cfg_problem(const ts_kernel_cfg& c, int batched) {
  if (c.block < 64 || c.block > 1024 || c.block % 64) return "block must be 64..1024, a multiple of 64";
  if (c.unroll != 1 && c.unroll != 2 && c.unroll != 4 && c.unroll != 8) return "unroll must be 1, 2, 4 or 8";
  if (batched) {
    const int P = c.wgs_per_tile;
    if (P < 0 || P > 128 || (P & (P - 1))) return "wgs_per_tile must be 1 (0 = 1) or a power of two up to 128";
    if (P > 1) {
      if (c.vec_bytes != 16 && c.vec_bytes != 8) return "workgroups sharing a tile use 16- or 8-byte vectors";
      if (c.block != 64 || c.unroll != 1 || c.grid_per_cu != 0 || c.tiles_per_wg > 1 || c.record_ahead != 0)
        return "workgroups sharing a tile take block 64, unroll 1, grid_per_cu 0, tiles_per_wg 1, record_ahead 0";
    } else if (c.vec_bytes != 16) {
      return "batched kernels with one workgroup per tile use 16-byte vectors";
    }
    if (c.grid_per_cu < 0 || c.grid_per_cu > 64) return "batched grid_per_cu must be 0..64";
    if (c.tile_elems < 0 || c.tile_elems % 8) return "tile_elems must be a multiple of 8";
    if (c.tiles_per_wg != 0 && c.tiles_per_wg != 1 && c.tiles_per_wg != 2 && c.tiles_per_wg != 4 &&
        c.tiles_per_wg != 8)
      return "tiles_per_wg must be 1, 2, 4 or 8 (0 = 1)";
    if (c.tiles_per_wg > 1 && c.unroll > 2) return "several tiles per workgroup take unroll 1 or 2";
    if (c.record_ahead != 0 && c.record_ahead != 1) return "record_ahead must be 0 or 1";
    if (c.record_ahead && (c.grid_per_cu != 0 || c.tiles_per_wg > 1))
      return "record_ahead needs one workgroup per tile (grid_per_cu 0, tiles_per_wg 1)";
  } else {
    if (c.vec_bytes != 16 && c.vec_bytes != 8 && c.vec_bytes != 4 && c.vec_bytes != 2)
      return "vec_bytes must be 16, 8, 4 or 2";
    if (c.grid_per_cu < 0 || c.grid_per_cu > 64) return "grid_per_cu must be 0..64";
    if (c.tiles_per_wg != 0 && c.tiles_per_wg != 1) return "plain kernels take tiles_per_wg 0 or 1";
    if (c.record_ahead != 0) return "plain kernels take record_ahead 0";
    if (c.wgs_per_tile != 0 && c.wgs_per_tile != 1) return "plain kernels take wgs_per_tile 0 or 1";
  }
  if ((c.nt_load != 0 && c.nt_load != 1) || (c.nt_store != 0 && c.nt_store != 1))
    return "nt flags must be 0 or 1";
  return "";
}

std::vector<ts_kernel_cfg> candidates(int batched) {
  std::vector<ts_kernel_cfg> out;
  if (!batched) {
    for (int vb : {16, 8})
      for (int block : {64, 128, 256, 512, 1024})
        for (int u : {1, 2, 4, 8})
          for (int ntl : {0, 1})
            for (int nts : {0, 1})
              for (int g : {0, 2, 4, 8}) {
                if (vb == 8 && g == 2) continue;  // keep the 8-byte set small
                // Workgroups of one or two waves only as one pass over the
                // array: a persistent grid of them leaves each CU a few waves.
                if (block < 256 && g != 0) continue;
                out.push_back(ts_kernel_cfg{block, u, vb, ntl, nts, g, 0, 1, 0, 1});
              }
  } else {
    // One workgroup per tile (grid_per_cu 0) with small tiles ...
    for (int block : {256, 512, 1024})
      for (int u : {1, 2})
        for (int ntl : {0, 1})
          for (int64_t tile : {512, 1024, 2048, 4096, 8192})
            for (int ahead : {0, 1})
              out.push_back(ts_kernel_cfg{block, u, 16, ntl, 1, 0, tile, 1, ahead, 1});
    // ... one-wave workgroups sharing each tile, one piece each ...
    for (int vb : {16, 8})
      for (int P : {8, 16, 32})
        for (int64_t tile : {1024, 2048, 4096})
          out.push_back(ts_kernel_cfg{64, 1, vb, 1, 1, 0, tile, 1, 0, P});
    // ... several consecutive small tiles per workgroup, all their first
    // loads in flight together ...
    for (int block : {256, 512})
      for (int u : {1, 2})
        for (int ntl : {0, 1})
          for (int k : {2, 4, 8})
            for (int64_t tile : {512, 1024, 2048})
              out.push_back(ts_kernel_cfg{block, u, 16, ntl, 1, 0, tile, k, 0, 1});
    // ... and persistent grids that stride over larger tiles.
    for (int block : {512, 1024})
      for (int u : {4, 8})
        for (int ntl : {0, 1})
          for (int g : {4, 8})
            for (int64_t tile : {16384, 65536})
              out.push_back(ts_kernel_cfg{block, u, 16, ntl, 1, g, tile, 1, 0, 1});
  }
  return out;
}

ts_kernel_cfg TuneTable::lookup(int op, int dtype, uint64_t n, int align, int batched) const {
  std::lock_guard<std::mutex> lk(mu_);
  const int b = batched ? 1 : 0;
  if (op >= 0 && op < 4 && dtype >= 0 && dtype < 4 && forced_set_[op][dtype][b])
    return forced_[op][dtype][b];
  const int bucket = size_bucket(n);
  auto it = entries_.find(TuneKey{op, dtype, bucket, align, b});
  if (it != entries_.end()) return it->second.cfg;
  const TuneEntry* best = nullptr;
  int best_dist = 1 << 30;
  for (const auto& kv : entries_) {
    const TuneKey& k = kv.first;
    if (k.op != op || k.dtype != dtype || k.align != align || k.batched != b) continue;
    const int dist = k.bucket > bucket ? k.bucket - bucket : bucket - k.bucket;
    if (dist < best_dist) {
      best_dist = dist;
      best = &kv.second;
    }
  }
  if (best) return best->cfg;
  ts_kernel_cfg c = default_cfg(b, dtype);
  if (align == TS_ALIGN_MIXED && !b) c.vec_bytes = 0;  // caller substitutes the element size
  return c;
}

void TuneTable::put(const TuneKey& k, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(mu_);
  entries_[k] = e;
}

void TuneTable::force(int op, int dtype, int batched, const ts_kernel_cfg* cfg) {
  std::lock_guard<std::mutex> lk(mu_);
  const int b = batched ? 1 : 0;
  forced_set_[op][dtype][b] = cfg != nullptr;
  if (cfg) forced_[op][dtype][b] = *cfg;
}

void TuneTable::clear() {
  std::lock_guard<std::mutex> lk(mu_);
  entries_.clear();
}

std::string TuneTable::to_json() const {
  std::lock_guard<std::mutex> lk(mu_);
  std::ostringstream os;
  os << "{\n  \"format\": \"tstream-tune\",\n  \"version\": " << kFormatVersion << ",\n  \"entries\": [";
  bool first = true;
  for (const auto& kv : entries_) {
    const TuneKey& k = kv.first;
    const ts_kernel_cfg& c = kv.second.cfg;
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "%s\n    {\"op\": \"%s\", \"dtype\": \"%s\", \"bucket\": %d, \"align\": %d, "
                  "\"batched\": %d, \"block\": %d, \"unroll\": %d, \"vec_bytes\": %d, "
                  "\"nt_load\": %d, \"nt_store\": %d, \"grid_per_cu\": %d, \"tile_elems\": %lld, "
                  "\"tiles_per_wg\": %d, \"record_ahead\": %d, \"wgs_per_tile\": %d, \"bytes_per_s\": %.6e}",
                  first ? "" : ",", kOpNames[k.op], kTypeNames[k.dtype], k.bucket, k.align,
                  k.batched, c.block, c.unroll, c.vec_bytes, c.nt_load, c.nt_store, c.grid_per_cu,
                  static_cast<long long>(c.tile_elems), c.tiles_per_wg, c.record_ahead,
                  c.wgs_per_tile < 1 ? 1 : c.wgs_per_tile, kv.second.bytes_per_s);
    os << buf;
    first = false;
  }
  os << "\n  ]\n}\n";
  return os.str();
}

// ---------------------------------------------------------------------------
// A small JSON reader for the table's own format: one object with "format",
// "version" and "entries" (an array of flat objects of strings and numbers).
// ---------------------------------------------------------------------------
namespace {

struct Reader {
  const std::string& s;
  size_t i = 0;
  std::string err;

  explicit Reader(const std::string& text) : s(text) {}

  void ws() {
    while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool fail(const std::string& m) {
    if (err.empty()) err = m + " at byte " + std::to_string(i);
    return false;
  }
  bool string(std::string& out) {
    ws();
    if (i >= s.size() || s[i] != '"') return fail("expected a string");
    ++i;
    out.clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') return fail("escapes are not used by this format");
      out.push_back(s[i++]);
    }
    if (i >= s.size()) return fail("unterminated string");
    ++i;
    return true;
  }
  bool number(double& out) {
    ws();
    const char* start = s.c_str() + i;
    char* end = nullptr;
    out = std::strtod(start, &end);
    if (end == start) return fail("expected a number");
    i += static_cast<size_t>(end - start);
    return true;
  }
  // value: string or number (kept as text/number)
  bool value(std::string& sv, double& nv, bool& is_str) {
    ws();
    if (i < s.size() && s[i] == '"') {
      is_str = true;
      return string(sv);
    }
    is_str = false;
    return number(nv);
  }
};

bool parse_entry(Reader& r, TuneKey& k, TuneEntry& e) {
  if (!r.eat('{')) return r.fail("expected an entry object");
  std::map<std::string, double> nums;
  std::map<std::string, std::string> strs;
  if (!r.eat('}')) {
    for (;;) {
      std::string key, sv;
      double nv = 0;
      bool is_str = false;
      if (!r.string(key)) return false;
      if (!r.eat(':')) return r.fail("expected ':'");
      if (!r.value(sv, nv, is_str)) return false;
      if (is_str) strs[key] = sv;
      else nums[key] = nv;
      if (r.eat(',')) continue;
      if (r.eat('}')) break;
      return r.fail("expected ',' or '}'");
    }
  }
  const char* need[] = {"bucket", "align", "batched", "block", "unroll", "vec_bytes",
                        "nt_load", "nt_store", "grid_per_cu", "tile_elems"};
  for (const char* n : need)
    if (!nums.count(n)) return r.fail(std::string("entry lacks \"") + n + "\"");
  if (!strs.count("op") || !strs.count("dtype")) return r.fail("entry lacks op or dtype");
  k.op = index_of(kOpNames, 4, strs["op"]);
  k.dtype = index_of(kTypeNames, 4, strs["dtype"]);
  if (k.op < 0 || k.dtype < 0) return r.fail("unknown op or dtype");
  k.bucket = static_cast<int>(nums["bucket"]);
  k.align = static_cast<int>(nums["align"]);
  k.batched = static_cast<int>(nums["batched"]) ? 1 : 0;
  if (k.bucket < 0 || k.bucket > 63 || k.align < 0 || k.align > 2) return r.fail("bad bucket or align");
  e.cfg.block = static_cast<int32_t>(nums["block"]);
  e.cfg.unroll = static_cast<int32_t>(nums["unroll"]);
  e.cfg.vec_bytes = static_cast<int32_t>(nums["vec_bytes"]);
  e.cfg.nt_load = static_cast<int32_t>(nums["nt_load"]);
  e.cfg.nt_store = static_cast<int32_t>(nums["nt_store"]);
  e.cfg.grid_per_cu = static_cast<int32_t>(nums["grid_per_cu"]);
  e.cfg.tile_elems = static_cast<int64_t>(nums["tile_elems"]);
  // Tables written before the field existed hold one tile per workgroup.
  e.cfg.tiles_per_wg = nums.count("tiles_per_wg") ? static_cast<int32_t>(nums["tiles_per_wg"]) : 1;
  e.cfg.record_ahead = nums.count("record_ahead") ? static_cast<int32_t>(nums["record_ahead"]) : 0;
  e.cfg.wgs_per_tile = nums.count("wgs_per_tile") ? static_cast<int32_t>(nums["wgs_per_tile"]) : 1;
  e.bytes_per_s = nums.count("bytes_per_s") ? nums["bytes_per_s"] : 0.0;
  const std::string why = cfg_problem(e.cfg, k.batched);
  if (!why.empty()) return r.fail("invalid configuration: " + why);
  return true;
}

}  // namespace

int TuneTable::from_json(const std::string& text, std::string* err) {
  Reader r(text);
  std::map<TuneKey, TuneEntry> parsed;
  std::string format;
  double version = -1;
  bool ok = r.eat('{');
  if (!ok) r.fail("expected '{'");
  bool have_entries = false;
  while (ok) {
    std::string key;
    if (!(ok = r.string(key))) break;
    if (!(ok = r.eat(':'))) {
      r.fail("expected ':'");
      break;
    }
    if (key == "format") {
      ok = r.string(format);
    } else if (key == "version") {
      ok = r.number(version);
    } else if (key == "entries") {
      have_entries = true;
      if (!(ok = r.eat('['))) {
        r.fail("expected '['");
        break;
      }
      if (!r.eat(']')) {
        for (;;) {
          TuneKey k{};
          TuneEntry e{};
          if (!(ok = parse_entry(r, k, e))) break;
          parsed[k] = e;
          if (r.eat(',')) continue;
          if (r.eat(']')) break;
          ok = r.fail("expected ',' or ']'");
          break;
        }
      }
    } else {
      ok = r.fail("unknown key \"" + key + "\"");
    }
    if (!ok) break;
    if (r.eat(',')) continue;
    if (r.eat('}')) break;
    ok = r.fail("expected ',' or '}'");
  }
  if (ok) {
    r.ws();
    if (r.i != text.size()) ok = r.fail("trailing data");
  }
  if (ok && format != "tstream-tune") ok = r.fail("not a tstream tuning file");
  if (ok && static_cast<int>(version) != kFormatVersion)
    ok = r.fail("format version " + std::to_string(static_cast<int>(version)) + " is not " +
                std::to_string(kFormatVersion));
  if (ok && !have_entries) ok = r.fail("no entries");
  if (!ok) {
    if (err) *err = r.err;
    return -1;
  }
  std::lock_guard<std::mutex> lk(mu_);
  for (const auto& kv : parsed) entries_[kv.first] = kv.second;
  return 0;
}

int TuneTable::load(const std::string& path, std::string* err) {
  std::ifstream f(path, std::ios::binary);
  if (!f) {
    if (err) *err = "cannot open " + path;
    return -1;
  }
  std::ostringstream ss;
  ss << f.rdbuf();
  std::string e;
  if (from_json(ss.str(), &e) != 0) {
    if (err) *err = path + ": " + e;
    return -1;
  }
  return 0;
}

int TuneTable::save(const std::string& path, std::string* err) const {
  const std::string text = to_json();
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) {
      if (err) *err = "cannot write " + tmp;
      return -1;
    }
    f << text;
    if (!f) {
      if (err) *err = "write failed: " + tmp;
      return -1;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    if (err) *err = "cannot rename " + tmp + " to " + path;
    return -1;
  }
  return 0;
}

TuneTable& tune_table() {
  static TuneTable t;
  return t;
}

}  // namespace ts
