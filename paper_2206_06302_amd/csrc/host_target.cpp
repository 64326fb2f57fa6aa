// host_target.cpp -- pinned worker pool, NUMA discovery and the element-wise
// maps of the host-CPU target (the paper's NUMA back-end, Section 4.1: CPU
// sets as targets, bytes divided evenly over them, work pinned to the cores
// that own the data).
#include "host_target.hpp"

#include <dirent.h>
#include <immintrin.h>
#include <pthread.h>
#include <sched.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <set>
#include <sstream>

namespace ts {

// ---------------------------------------------------------------------------
// Worker pool
// ---------------------------------------------------------------------------
HostPool::HostPool(const std::vector<int>& cpus) : cpus_(cpus) {
  threads_.reserve(cpus_.size());
  for (int w = 0; w < static_cast<int>(cpus_.size()); ++w) threads_.emplace_back([this, w] { worker(w); });
}

HostPool::~HostPool() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_go_.notify_all();
  for (auto& t : threads_) t.join();
}

void HostPool::worker(int w) {
  if (cpus_[w] >= 0) {  // best effort: an unpinnable CPU leaves the thread floating
    cpu_set_t one;
    CPU_ZERO(&one);
    CPU_SET(cpus_[w], &one);
    pthread_setaffinity_np(pthread_self(), sizeof one, &one);
  }
  uint64_t seen = 0;
  for (;;) {
    const std::function<void(int)>* job;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_go_.wait(lk, [&] { return stop_ || generation_ != seen; });
      if (stop_) return;
      seen = generation_;
      job = job_;
    }
    (*job)(w);
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) cv_done_.notify_all();
    }
  }
}

void HostPool::run(const std::function<void(int)>& f) {
  std::lock_guard<std::mutex> serial(run_mu_);
  std::unique_lock<std::mutex> lk(mu_);
  job_ = &f;
  pending_ = size();
  ++generation_;
  cv_go_.notify_all();
  cv_done_.wait(lk, [&] { return pending_ == 0; });
  job_ = nullptr;
}

// ---------------------------------------------------------------------------
// Topology
// ---------------------------------------------------------------------------
std::vector<int> host_allowed_cpus() {
  cpu_set_t set;
  CPU_ZERO(&set);
  std::vector<int> out;
  if (sched_getaffinity(0, sizeof set, &set) == 0) {
    for (int c = 0; c < CPU_SETSIZE; ++c)
      if (CPU_ISSET(c, &set)) out.push_back(c);
  }
  return out;
}

namespace {
// "0-3,8,10-11" -> {0,1,2,3,8,10,11}
std::vector<int> parse_cpulist(const std::string& s) {
  std::vector<int> out;
  std::stringstream ss(s);
  std::string item;
  while (std::getline(ss, item, ',')) {
    if (item.empty() || item == "\n") continue;
    int a = 0, b = 0;
    if (std::sscanf(item.c_str(), "%d-%d", &a, &b) == 2) {
      for (int c = a; c <= b; ++c) out.push_back(c);
    } else if (std::sscanf(item.c_str(), "%d", &a) == 1) {
      out.push_back(a);
    }
  }
  return out;
}
}  // namespace

std::vector<std::vector<int>> host_domains() {
  const std::vector<int> allowed = host_allowed_cpus();
  const std::set<int> ok(allowed.begin(), allowed.end());
  std::vector<std::pair<int, std::vector<int>>> nodes;
  if (DIR* d = opendir("/sys/devices/system/node")) {
    while (dirent* e = readdir(d)) {
      int id = -1;
      if (std::sscanf(e->d_name, "node%d", &id) != 1 || id < 0) continue;
      std::ifstream f(std::string("/sys/devices/system/node/") + e->d_name + "/cpulist");
      std::string line;
      if (!std::getline(f, line)) continue;
      std::vector<int> cpus;
      for (int c : parse_cpulist(line))
        if (ok.count(c)) cpus.push_back(c);
      if (!cpus.empty()) nodes.emplace_back(id, cpus);
    }
    closedir(d);
  }
  std::sort(nodes.begin(), nodes.end());
  std::vector<std::vector<int>> out;
  for (auto& n : nodes) out.push_back(n.second);
  if (out.empty() && !allowed.empty()) out.push_back(allowed);
  return out;
}

// ---------------------------------------------------------------------------
// Element-wise maps (Section 5, Listing 4), one contiguous block each.
// ---------------------------------------------------------------------------
namespace {

template <class T>
void map_plain(int op, const T* x, const T* y, T* d, uint64_t lo, uint64_t hi, T q) {
  switch (op) {
    case 0:
      for (uint64_t j = lo; j < hi; ++j) d[j] = x[j];
      break;
    case 1:
      for (uint64_t j = lo; j < hi; ++j) d[j] = q * x[j];
      break;
    case 2:
      for (uint64_t j = lo; j < hi; ++j) d[j] = x[j] + y[j];
      break;
    default:
      for (uint64_t j = lo; j < hi; ++j) d[j] = std::fma(q, y[j], x[j]);
      break;
  }
}

// The same loops compiled for AVX2 + FMA3, so the fused multiply-add is one
// instruction instead of a library call (selected at run time).
template <class T>
__attribute__((target("avx2,fma"))) void map_fma(int op, const T* x, const T* y, T* d, uint64_t lo,
                                                 uint64_t hi, T q) {
  switch (op) {
    case 0:
      for (uint64_t j = lo; j < hi; ++j) d[j] = x[j];
      break;
    case 1:
      for (uint64_t j = lo; j < hi; ++j) d[j] = q * x[j];
      break;
    case 2:
      for (uint64_t j = lo; j < hi; ++j) d[j] = x[j] + y[j];
      break;
    default:
      for (uint64_t j = lo; j < hi; ++j) d[j] = __builtin_fma(q, y[j], x[j]);
      break;
  }
}

template <>
__attribute__((target("avx2,fma"))) void map_fma<float>(int op, const float* x, const float* y, float* d,
                                                        uint64_t lo, uint64_t hi, float q) {
  switch (op) {
    case 0:
      for (uint64_t j = lo; j < hi; ++j) d[j] = x[j];
      break;
    case 1:
      for (uint64_t j = lo; j < hi; ++j) d[j] = q * x[j];
      break;
    case 2:
      for (uint64_t j = lo; j < hi; ++j) d[j] = x[j] + y[j];
      break;
    default:
      for (uint64_t j = lo; j < hi; ++j) d[j] = __builtin_fmaf(q, y[j], x[j]);
      break;
  }
}

// Large blocks: the same arithmetic with 32-byte streaming stores, which
// write whole lines without first reading them (STREAM's destination is
// not read again by the map).  Head and tail run element by element; the
// sfence orders the streaming stores before the worker reports completion.
constexpr uint64_t kStreamBytes = 1u << 20;  // smaller blocks stay in cache

__attribute__((target("avx2,fma"))) void map_stream_f64(int op, const double* x, const double* y, double* d,
                                                        uint64_t lo, uint64_t hi, double q) {
  uint64_t j = lo;
  for (; j < hi && (reinterpret_cast<uintptr_t>(d + j) & 31); ++j)  // head up to 32-byte alignment
    d[j] = op == 0 ? x[j] : op == 1 ? q * x[j] : op == 2 ? x[j] + y[j] : __builtin_fma(q, y[j], x[j]);
  const __m256d vq = _mm256_set1_pd(q);
  for (; j + 4 <= hi; j += 4) {
    const __m256d a = _mm256_loadu_pd(x + j);
    __m256d r;
    if (op == 0) r = a;
    else if (op == 1) r = _mm256_mul_pd(vq, a);
    else if (op == 2) r = _mm256_add_pd(a, _mm256_loadu_pd(y + j));
    else r = _mm256_fmadd_pd(vq, _mm256_loadu_pd(y + j), a);
    _mm256_stream_pd(d + j, r);
  }
  for (; j < hi; ++j)
    d[j] = op == 0 ? x[j] : op == 1 ? q * x[j] : op == 2 ? x[j] + y[j] : __builtin_fma(q, y[j], x[j]);
  _mm_sfence();
}

__attribute__((target("avx2,fma"))) void map_stream_f32(int op, const float* x, const float* y, float* d,
                                                        uint64_t lo, uint64_t hi, float q) {
  uint64_t j = lo;
  for (; j < hi && (reinterpret_cast<uintptr_t>(d + j) & 31); ++j)
    d[j] = op == 0 ? x[j] : op == 1 ? q * x[j] : op == 2 ? x[j] + y[j] : __builtin_fmaf(q, y[j], x[j]);
  const __m256 vq = _mm256_set1_ps(q);
  for (; j + 8 <= hi; j += 8) {
    const __m256 a = _mm256_loadu_ps(x + j);
    __m256 r;
    if (op == 0) r = a;
    else if (op == 1) r = _mm256_mul_ps(vq, a);
    else if (op == 2) r = _mm256_add_ps(a, _mm256_loadu_ps(y + j));
    else r = _mm256_fmadd_ps(vq, _mm256_loadu_ps(y + j), a);
    _mm256_stream_ps(d + j, r);
  }
  for (; j < hi; ++j)
    d[j] = op == 0 ? x[j] : op == 1 ? q * x[j] : op == 2 ? x[j] + y[j] : __builtin_fmaf(q, y[j], x[j]);
  _mm_sfence();
}

bool cpu_has_fma() {
  static const bool has = __builtin_cpu_supports("fma") && __builtin_cpu_supports("avx2");
  return has;
}

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

template <class T>
HostPart checksum_block(const T* x, uint64_t lo, uint64_t hi, double e) {
  HostPart p{0.0, 0.0, std::nan(""), 0};
  uint64_t ebits;
  std::memcpy(&ebits, &e, 8);
  for (uint64_t j = lo; j < hi; ++j) {
    const double v = static_cast<double>(x[j]);
    const double dv = std::fabs(v - e);
    p.sum += v;
    p.absdev += dv;
    p.maxdev = std::fmax(p.maxdev, dv);
    uint64_t vb;
    std::memcpy(&vb, &v, 8);
    if (vb != ebits && !(std::isnan(v) && std::isnan(e))) ++p.mism;
  }
  return p;
}

}  // namespace

void host_map_f64(int op, const double* x, const double* y, double* d, uint64_t lo, uint64_t hi, double q) {
  if (!cpu_has_fma()) map_plain<double>(op, x, y, d, lo, hi, q);
  else if ((hi - lo) * sizeof(double) >= kStreamBytes) map_stream_f64(op, x, y, d, lo, hi, q);
  else map_fma<double>(op, x, y, d, lo, hi, q);
}

void host_map_f32(int op, const float* x, const float* y, float* d, uint64_t lo, uint64_t hi, float q) {
  if (!cpu_has_fma()) map_plain<float>(op, x, y, d, lo, hi, q);
  else if ((hi - lo) * sizeof(float) >= kStreamBytes) map_stream_f32(op, x, y, d, lo, hi, q);
  else map_fma<float>(op, x, y, d, lo, hi, q);
}

namespace {

// Constant fill of a large block with 32-byte streaming stores (the owning
// worker still touches every page first).
template <class T>
__attribute__((target("avx2"))) void fill_stream(T* d, uint64_t lo, uint64_t hi, T v) {
  uint64_t j = lo;
  for (; j < hi && (reinterpret_cast<uintptr_t>(d + j) & 31); ++j) d[j] = v;
  constexpr uint64_t E = 32 / sizeof(T);
  __m256i pattern;
  T lanes[E];
  for (uint64_t e = 0; e < E; ++e) lanes[e] = v;
  std::memcpy(&pattern, lanes, 32);
  for (; j + E <= hi; j += E) _mm256_stream_si256(reinterpret_cast<__m256i*>(d + j), pattern);
  for (; j < hi; ++j) d[j] = v;
  _mm_sfence();
}

}  // namespace

void host_fill_f64(double* d, uint64_t lo, uint64_t hi, double v) {
  if (cpu_has_fma() && (hi - lo) * sizeof(double) >= kStreamBytes) return fill_stream(d, lo, hi, v);
  for (uint64_t j = lo; j < hi; ++j) d[j] = v;
}

void host_fill_f32(float* d, uint64_t lo, uint64_t hi, float v) {
  if (cpu_has_fma() && (hi - lo) * sizeof(float) >= kStreamBytes) return fill_stream(d, lo, hi, v);
  for (uint64_t j = lo; j < hi; ++j) d[j] = v;
}

// vlo + w * u01, u01 = (h >> 11) * 2^-53, with separate roundings.
static double uniform_range_at(uint64_t state0, uint64_t counter, double vlo, double w) {
  const double u01 = static_cast<double>(mix64(state0 + counter * kGamma) >> 11) * 0x1p-53;
  const double scaled = w * u01;
  return vlo + scaled;
}

void host_fill_uniform_f64(double* d, uint64_t lo, uint64_t hi, uint64_t state0, uint64_t first, double vlo,
                           double w) {
  for (uint64_t j = lo; j < hi; ++j) d[j] = uniform_range_at(state0, first + j + 1, vlo, w);
}

void host_fill_uniform_f32(float* d, uint64_t lo, uint64_t hi, uint64_t state0, uint64_t first, double vlo,
                           double w) {
  for (uint64_t j = lo; j < hi; ++j) d[j] = static_cast<float>(uniform_range_at(state0, first + j + 1, vlo, w));
}

HostPart host_checksum_f64(const double* x, uint64_t lo, uint64_t hi, double expected) {
  return checksum_block(x, lo, hi, expected);
}

HostPart host_checksum_f32(const float* x, uint64_t lo, uint64_t hi, double expected) {
  return checksum_block(x, lo, hi, expected);
}

uint64_t host_mismatch(const void* x, const void* r, uint64_t lo, uint64_t hi, size_t es, bool is_f64) {
  uint64_t count = 0;
  const char* xb = static_cast<const char*>(x);
  const char* rb = static_cast<const char*>(r);
  for (uint64_t j = lo; j < hi; ++j) {
    if (std::memcmp(xb + j * es, rb + j * es, es) == 0) continue;
    double a, b;
    if (is_f64) {
      std::memcpy(&a, xb + j * es, 8);
      std::memcpy(&b, rb + j * es, 8);
    } else {
      float fa, fb;
      std::memcpy(&fa, xb + j * es, 4);
      std::memcpy(&fb, rb + j * es, 4);
      a = fa;
      b = fb;
    }
    if (std::isnan(a) && std::isnan(b)) continue;
    ++count;
  }
  return count;
}

}  // namespace ts
