// Sanitizer driver for the GPU-free host code of the library (built with
// g++ -fsanitize=... by tests/test_sanitizers.py; test infrastructure only):
// the tuning-file parser on mutated inputs, the plain and batch planners on
// random inputs, and the pinned worker pool under repeated fork-join runs.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "host_target.hpp"
#include "ts_layout.hpp"
#include "tune.hpp"

int main(int argc, char** argv) {
  const int fuzz = argc > 1 ? std::atoi(argv[1]) : 20000;
  const int plans = argc > 2 ? std::atoi(argv[2]) : 5000;
  const int runs = argc > 3 ? std::atoi(argv[3]) : 500;
  std::mt19937_64 rng(42);
  const std::string good =
      "{\"format\": \"tstream-tune\", \"version\": 1, \"entries\": [{\"op\": \"triad\", \"dtype\": \"f64\", "
      "\"bucket\": 27, \"align\": 0, \"batched\": 0, \"block\": 256, \"unroll\": 1, \"vec_bytes\": 16, "
      "\"nt_load\": 1, \"nt_store\": 1, \"grid_per_cu\": 0, \"tile_elems\": 0, \"bytes_per_s\": 6.5e12}]}";
  int accepted = 0;
  for (int it = 0; it < fuzz; ++it) {
    std::string s = good;
    const int muts = 1 + static_cast<int>(rng() % 4);
    for (int m = 0; m < muts; ++m) {
      const size_t pos = rng() % (s.size() + 1);
      switch (rng() % 4) {
        case 0:
          if (pos < s.size()) s.erase(pos, 1 + rng() % 8);
          break;
        case 1: s.insert(pos, 1, static_cast<char>(rng() % 256)); break;
        case 2:
          if (pos < s.size()) s[pos] = static_cast<char>(rng() % 256);
          break;
        default: s = s.substr(0, pos); break;
      }
    }
    ts::TuneTable t;
    std::string err;
    if (t.from_json(s, &err) == 0) ++accepted;
    (void)t.lookup(3, 0, 1ull << 27, 0, 0);
  }
  std::printf("parser: %d of %d mutated tables accepted\n", accepted, fuzz);
  for (int it = 0; it < plans; ++it) {
    const size_t es = std::vector<size_t>{8, 4, 2, 1}[rng() % 4];
    const size_t count = rng() % 20;
    std::vector<ts::HostDesc> d(count);
    for (auto& h : d) {
      const uintptr_t base = (1ull << 30) + (rng() % 1000) * 4096;
      h = ts::HostDesc{base + (rng() % 16) / es * es, base + (1ull << 28) + (rng() % 16) / es * es,
                       base + (2ull << 28) + (rng() % 16) / es * es, rng() % 5000, 1.5};
    }
    std::vector<ts::BatchDesc> bd;
    std::vector<ts::BatchTile> bt;
    uint64_t total = 0;
    std::string err;
    const int64_t tile = 8 * static_cast<int64_t>(1 + rng() % 300);
    if (ts::plan_batch(d.data(), count, es, tile, bd, bt, total, err) != 0) {
      std::printf("batch plan failed: %s\n", err.c_str());
      return 1;
    }
    uint64_t covered = 0;
    for (const auto& t : bt) covered += t.count;
    if (covered != total) {
      std::printf("batch plan covers %llu of %llu\n", static_cast<unsigned long long>(covered),
                  static_cast<unsigned long long>(total));
      return 1;
    }
    const uintptr_t x = 4096 + (rng() % 128) / es * es, y = 8192 + (rng() % 128) / es * es,
                    z = 12288 + (rng() % 128) / es * es;
    const uint64_t n = rng() % 1000;
    ts::PlainPlan p{};
    for (size_t vb : {16, 8, 4, 2})
      if (vb >= es && ts::plan_plain(x, &y, z, n, es, vb, p) && p.head + p.nvec * (vb / es) + p.tail != n) {
        std::printf("plain plan does not cover n\n");
        return 1;
      }
  }
  std::printf("planners: %d random cases\n", plans);
  std::vector<int> cpus = ts::host_allowed_cpus();
  if (cpus.size() > 8) cpus.resize(8);
  for (int rep = 0; rep < 2; ++rep) {
    ts::HostPool pool(cpus);
    std::vector<double> v(1 << 14, 0.0);
    for (int it = 0; it < runs; ++it)
      pool.run([&](int w) {
        uint64_t lo, hi;
        ts::HostPool::block(v.size(), pool.size(), w, &lo, &hi);
        for (uint64_t j = lo; j < hi; ++j) v[j] += 1.0;
      });
    for (double e : v)
      if (e != static_cast<double>(runs)) {
        std::printf("pool result wrong\n");
        return 1;
      }
  }
  std::printf("pool: %d fork-join runs on %zu workers\n", runs, cpus.size());
  return 0;
}
