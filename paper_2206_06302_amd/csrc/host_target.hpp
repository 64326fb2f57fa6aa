// host_target.hpp -- the host-CPU target of libtstream: a set of CPUs with
// one pinned worker thread each, arrays divided into equal contiguous blocks
// over the workers (the paper's NUMA block allocator and executor, Section
// 4.1).  Pure C++ (no HIP).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <condition_variable>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace ts {

// Fork-join pool of pinned workers.  run(f) calls f(w) on worker w for every
// worker and returns when all have finished; calls are serialised.
class HostPool {
 public:
  explicit HostPool(const std::vector<int>& cpus);
  ~HostPool();
  HostPool(const HostPool&) = delete;
  HostPool& operator=(const HostPool&) = delete;

  int size() const { return static_cast<int>(cpus_.size()); }
  const std::vector<int>& cpus() const { return cpus_; }
  void run(const std::function<void(int)>& f);
  // Contiguous block of worker w when n elements are divided evenly.
  static void block(uint64_t n, int workers, int w, uint64_t* lo, uint64_t* hi) {
    *lo = n * static_cast<uint64_t>(w) / static_cast<uint64_t>(workers);
    *hi = n * static_cast<uint64_t>(w + 1) / static_cast<uint64_t>(workers);
  }

 private:
  void worker(int w);
  std::vector<int> cpus_;
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::mutex run_mu_;
  std::condition_variable cv_go_, cv_done_;
  const std::function<void(int)>* job_ = nullptr;
  uint64_t generation_ = 0;
  int pending_ = 0;
  bool stop_ = false;
};

// NUMA domains of this machine restricted to the CPUs the process may use
// (one domain holding every allowed CPU when the topology is not exposed).
std::vector<std::vector<int>> host_domains();
std::vector<int> host_allowed_cpus();

// Element-wise maps over [lo, hi) (binary64 or binary32 storage).
void host_map_f64(int op, const double* x, const double* y, double* d, uint64_t lo, uint64_t hi, double q);
void host_map_f32(int op, const float* x, const float* y, float* d, uint64_t lo, uint64_t hi, float q);
void host_fill_f64(double* d, uint64_t lo, uint64_t hi, double v);
void host_fill_f32(float* d, uint64_t lo, uint64_t hi, float v);
// Elements [lo, hi) of the uniform fill over [vlo, vlo + w).
void host_fill_uniform_f64(double* d, uint64_t lo, uint64_t hi, uint64_t state0, uint64_t first, double vlo,
                           double w);
void host_fill_uniform_f32(float* d, uint64_t lo, uint64_t hi, uint64_t state0, uint64_t first, double vlo,
                           double w);

struct HostPart {
  double sum, absdev, maxdev;
  uint64_t mism;
};
HostPart host_checksum_f64(const double* x, uint64_t lo, uint64_t hi, double expected);
HostPart host_checksum_f32(const float* x, uint64_t lo, uint64_t hi, double expected);
uint64_t host_mismatch(const void* x, const void* r, uint64_t lo, uint64_t hi, size_t es, bool is_f64);

}  // namespace ts
