// transform.cpp -- element-wise transforms with a user expression, compiled
// at run time with hipRTC for the target's GPU.
//
// The paper's GPU executor runs any device callable (Section 4.2), and its
// hello-world example transforms a vector of chars with to_upper (Section
// 3.4, Listing 3).  A C ABI cannot carry a callable, so the callable arrives
// as the text of a C++ expression in x, y and q; the library wraps it in
// kernels (16- and 8-byte vectors for operands that share their alignment,
// and an element-wise fallback), compiles them once per (expression, inputs,
// storage type, architecture) and launches one on the executing target's
// stream.
// hipRTC is opened lazily (dlopen), so it is needed only when transforms
// are used.
#include <dlfcn.h>
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>

#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/tstream.h"
#include "host_transform.hpp"
#include "ts_handles.hpp"
#include "ts_layout.hpp"

using namespace ts;

namespace {

constexpr uint32_t kTransformMagic = 0x54524631u;

// The hipRTC entry points used here, resolved from the loaded library.
struct Rtc {
  hiprtcResult (*create)(hiprtcProgram*, const char*, const char*, int, const char**, const char**);
  hiprtcResult (*compile)(hiprtcProgram, int, const char**);
  hiprtcResult (*log_size)(hiprtcProgram, size_t*);
  hiprtcResult (*log)(hiprtcProgram, char*);
  hiprtcResult (*code_size)(hiprtcProgram, size_t*);
  hiprtcResult (*code)(hiprtcProgram, char*);
  hiprtcResult (*destroy)(hiprtcProgram*);
  const char* (*error_string)(hiprtcResult);
  bool ok = false;
  std::string why;
};

const Rtc& rtc() {
  static Rtc r = [] {
    Rtc x;
    void* h = dlopen("libhiprtc.so.7", RTLD_NOW | RTLD_GLOBAL);
    if (!h) h = dlopen("/opt/rocm/lib/libhiprtc.so.7", RTLD_NOW | RTLD_GLOBAL);
    if (!h) {
      x.why = std::string("hipRTC is not available: ") + dlerror();
      return x;
    }
    bool all = true;
    auto get = [&](auto& fn, const char* name) {
      fn = reinterpret_cast<std::remove_reference_t<decltype(fn)>>(dlsym(h, name));
      all = all && fn != nullptr;
    };
    get(x.create, "hiprtcCreateProgram");
    get(x.compile, "hiprtcCompileProgram");
    get(x.log_size, "hiprtcGetProgramLogSize");
    get(x.log, "hiprtcGetProgramLog");
    get(x.code_size, "hiprtcGetCodeSize");
    get(x.code, "hiprtcGetCode");
    get(x.destroy, "hiprtcDestroyProgram");
    get(x.error_string, "hiprtcGetErrorString");
    x.ok = all;
    if (!all) x.why = "hipRTC library lacks an expected entry point";
    return x;
  }();
  return r;
}

// Storage and arithmetic types of each storage format inside the generated
// source.  The 16-bit formats widen exactly to float and narrow by
// round-to-nearest-even, as the built-in kernels do.
struct TypeText {
  const char* storage;
  const char* arith;
  const char* widen;   // expression of `v` (storage) giving the arithmetic value
  const char* narrow;  // expression of `r` (arithmetic) giving the storage value
};

TypeText type_text(int dtype) {
  switch (dtype) {
    case TS_F64: return {"double", "double", "v", "r"};
    case TS_F32: return {"float", "float", "v", "r"};
    case TS_BF16:
      return {"unsigned short", "float", "__builtin_bit_cast(float, (unsigned int)v << 16)",
              "__builtin_bit_cast(unsigned short, (__bf16)ts_keep(r))"};
    case TS_F16:
      return {"unsigned short", "float", "(float)__builtin_bit_cast(_Float16, v)",
              "__builtin_bit_cast(unsigned short, (_Float16)ts_keep(r))"};
    default: return {"unsigned char", "int", "(int)v", "(unsigned char)(r)"};
  }
}

// The generated source holds three kernels around the expression:
//   ts_transform_vec     16-byte nontemporal vectors (16 / element size
//                        elements), one per lane in one pass (a grid-stride
//                        loop covers arrays beyond the largest launch), plus
//                        an element-wise head and tail, for operands that
//                        share their misalignment modulo 16 bytes;
//   ts_transform_vec8    the same with 8-byte vectors, for operands that share
//                        their misalignment modulo 8 bytes;
//   ts_transform_kernel  element-wise with a grid-stride loop, for any operands.
std::string kernel_source(const std::string& expr, int n_inputs, int dtype) {
  const TypeText t = type_text(dtype);
  const bool two = n_inputs == 2;
  std::string s;
  s += "typedef " + std::string(t.storage) + " ts_store_t;\n";
  s += "typedef " + std::string(t.arith) + " ts_arith_t;\n";
  s += "typedef unsigned int ts_u4 __attribute__((ext_vector_type(4)));\n";
  s += "typedef unsigned int ts_u2 __attribute__((ext_vector_type(2)));\n";
  s += "__device__ inline float ts_keep(float v) { asm(\"\" : \"+v\"(v)); return v; }\n";
  s += "__device__ inline ts_arith_t ts_widen(ts_store_t v) { return " + std::string(t.widen) + "; }\n";
  s += "__device__ inline ts_store_t ts_narrow(ts_arith_t r) { return " + std::string(t.narrow) + "; }\n";
  s += "__device__ inline ts_store_t ts_apply(ts_store_t xv, ts_store_t yv, ts_arith_t q) {\n"
       "  (void)q; (void)yv;\n"
       "  const ts_arith_t x = ts_widen(xv);\n";
  if (two) s += "  const ts_arith_t y = ts_widen(yv);\n";
  s += "  return ts_narrow((ts_arith_t)(" + expr + "));\n}\n";
  s += "extern \"C\" __global__ void ts_transform_kernel(const ts_store_t* __restrict__ xs,\n"
       "    const ts_store_t* __restrict__ ys, ts_store_t* ds, double qd, unsigned long long n) {\n"
       "  const ts_arith_t q = (ts_arith_t)qd;\n"
       "  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;\n"
       "  for (unsigned long long j = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; j < n;\n"
       "       j += stride)\n";
  s += two ? "    ds[j] = ts_apply(xs[j], ys[j], q);\n}\n" : "    ds[j] = ts_apply(xs[j], xs[j], q);\n}\n";
  // One vector kernel per width W: name, W-byte raw vector type, elements per vector.
  const struct { const char* name; const char* raw; const char* elems; } widths[] = {
      {"ts_transform_vec", "ts_u4", "(16 / sizeof(ts_store_t))"},
      {"ts_transform_vec8", "ts_u2", "(8 / sizeof(ts_store_t))"}};
  for (const auto& w : widths) {
    const std::string vt = std::string(w.name) + "_t";
    s += "struct " + vt + " { ts_store_t v[" + w.elems + "]; };\n";
    s += "extern \"C\" __global__ void " + std::string(w.name) + "(const ts_store_t* __restrict__ xs,\n"
         "    const ts_store_t* __restrict__ ys, ts_store_t* ds, double qd, unsigned long long head,\n"
         "    unsigned long long nvec, unsigned long long tail) {\n"
         "  const ts_arith_t q = (ts_arith_t)qd;\n"
         "  const unsigned long long g = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;\n"
         "  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;\n"
         "  const unsigned long long t0 = head + nvec * " + w.elems + ";\n";
    s += two ? "  if (g < head) ds[g] = ts_apply(xs[g], ys[g], q);\n"
               "  if (g < tail) ds[t0 + g] = ts_apply(xs[t0 + g], ys[t0 + g], q);\n"
             : "  if (g < head) ds[g] = ts_apply(xs[g], xs[g], q);\n"
               "  if (g < tail) ds[t0 + g] = ts_apply(xs[t0 + g], xs[t0 + g], q);\n";
    s += "  for (unsigned long long v = g; v < nvec; v += stride) {\n"
         "    const " + vt + " xv = __builtin_bit_cast(" + vt + ",\n"
         "        __builtin_nontemporal_load(reinterpret_cast<const " + w.raw + "*>(xs + head) + v));\n";
    s += two ? "    const " + vt + " yv = __builtin_bit_cast(" + vt + ",\n"
               "        __builtin_nontemporal_load(reinterpret_cast<const " + w.raw + "*>(ys + head) + v));\n"
             : "    const " + vt + " yv = xv;\n";
    s += "    " + vt + " dv;\n"
         "#pragma unroll\n"
         "    for (unsigned e = 0; e < " + w.elems + "; ++e) dv.v[e] = ts_apply(xv.v[e], yv.v[e], q);\n"
         "    __builtin_nontemporal_store(__builtin_bit_cast(" + w.raw + ", dv), reinterpret_cast<" + w.raw +
         "*>(ds + head) + v);\n"
         "  }\n}\n";
  }
  return s;
}

// Code objects already compiled, by (expression, inputs, type, architecture).
std::mutex g_cache_mu;
std::map<std::tuple<std::string, int, int, std::string>, std::shared_ptr<std::vector<char>>> g_code_cache;

}  // namespace

struct ts_transform_s {
  uint32_t magic;
  int device;
  int dtype;
  int n_inputs;
  hipModule_t module;
  hipFunction_t fn;      // element-wise, grid-stride
  hipFunction_t fn_vec;   // 16-byte vectors, one pass
  hipFunction_t fn_vec8;  // 8-byte vectors, one pass
  HostTransformFn host_fn;  // host-CPU targets: the compiled block function
  std::string log;
};

extern "C" {

int ts_transform_create(ts_target t, const char* expr, int n_inputs, ts_dtype dtype, ts_transform* out) {
  try {
    if (!ts_ok_target_handle(t) || !expr || !out) return api_fail(TS_E_INVALID, "invalid target, expression or out");
    if (n_inputs != 1 && n_inputs != 2) return api_fail(TS_E_INVALID, "n_inputs must be 1 or 2");
    if (dtype < TS_F64 || dtype > TS_U8) return api_fail(TS_E_INVALID, "unknown dtype");
    if (t->host) {
      if (dtype != TS_F64 && dtype != TS_F32 && dtype != TS_U8)
        return api_fail(TS_E_UNSUPPORTED, "host targets support binary64, binary32 and byte storage");
      HostTransformFn fn = nullptr;
      std::string log;
      const int st = host_transform_compile(expr, n_inputs, static_cast<int>(dtype), &fn, &log);
      if (st == TS_E_INVALID) return api_fail(st, "expression does not compile: %s", log.c_str());
      if (st != TS_OK) return api_fail(st, "%s", log.c_str());
      ts_transform_s* x = new ts_transform_s();
      x->device = t->device;
      x->dtype = dtype;
      x->n_inputs = n_inputs;
      x->host_fn = fn;
      x->log = log;
      x->magic = kTransformMagic;
      *out = x;
      return TS_OK;
    }
    const Rtc& r = rtc();
    if (!r.ok) return api_fail(TS_E_UNSUPPORTED, "%s", r.why.c_str());
    hipError_t he = hipSetDevice(t->device);
    if (he != hipSuccess) return api_hip_fail(he, "hipSetDevice");
    std::string arch = t->info.arch;
    const std::string arch_name = arch.substr(0, arch.find(':'));
    const auto key = std::make_tuple(std::string(expr), n_inputs, static_cast<int>(dtype), arch);
    std::shared_ptr<std::vector<char>> code;
    std::string log;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      auto it = g_code_cache.find(key);
      if (it != g_code_cache.end()) code = it->second;
    }
    if (!code) {
      const std::string src = kernel_source(expr, n_inputs, dtype);
      hiprtcProgram prog = nullptr;
      hiprtcResult rr = r.create(&prog, src.c_str(), "ts_transform.hip", 0, nullptr, nullptr);
      if (rr != HIPRTC_SUCCESS) return api_fail(TS_E_DEVICE, "hiprtcCreateProgram: %s", r.error_string(rr));
      const std::string arch_opt = "--offload-arch=" + arch_name;
      const char* opts[] = {arch_opt.c_str(), "-O3", "-ffp-contract=off", "-std=c++17",
                            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
      rr = r.compile(prog, 8, opts);
      size_t ls = 0;
      if (r.log_size(prog, &ls) == HIPRTC_SUCCESS && ls > 1) {
        log.resize(ls);
        r.log(prog, &log[0]);
        log.resize(std::strlen(log.c_str()));
      }
      if (rr != HIPRTC_SUCCESS) {
        r.destroy(&prog);
        return api_fail(TS_E_INVALID, "expression does not compile: %s", log.empty() ? r.error_string(rr) : log.c_str());
      }
      size_t cs = 0;
      rr = r.code_size(prog, &cs);
      auto buf = std::make_shared<std::vector<char>>(cs);
      if (rr == HIPRTC_SUCCESS) rr = r.code(prog, buf->data());
      r.destroy(&prog);
      if (rr != HIPRTC_SUCCESS) return api_fail(TS_E_DEVICE, "hiprtcGetCode: %s", r.error_string(rr));
      code = buf;
      std::lock_guard<std::mutex> lk(g_cache_mu);
      g_code_cache[key] = code;
    }
    hipModule_t mod = nullptr;
    he = hipModuleLoadData(&mod, code->data());
    if (he != hipSuccess) return api_hip_fail(he, "hipModuleLoadData");
    hipFunction_t fn = nullptr, fn_vec = nullptr, fn_vec8 = nullptr;
    he = hipModuleGetFunction(&fn, mod, "ts_transform_kernel");
    if (he == hipSuccess) he = hipModuleGetFunction(&fn_vec, mod, "ts_transform_vec");
    if (he == hipSuccess) he = hipModuleGetFunction(&fn_vec8, mod, "ts_transform_vec8");
    if (he != hipSuccess) {
      (void)hipModuleUnload(mod);
      return api_hip_fail(he, "hipModuleGetFunction");
    }
    ts_transform_s* x = new ts_transform_s();
    x->device = t->device;
    x->dtype = dtype;
    x->n_inputs = n_inputs;
    x->module = mod;
    x->fn = fn;
    x->fn_vec = fn_vec;
    x->fn_vec8 = fn_vec8;
    x->log = log;
    x->magic = kTransformMagic;
    *out = x;
    return TS_OK;
  } catch (...) {
    return api_fail(TS_E_OOM, "host allocation failed");
  }
}

int ts_transform_apply(ts_target t, ts_transform x, ts_array a, ts_array b, ts_array d, double q) {
  try {
    if (!ts_ok_target_handle(t) || !x || x->magic != kTransformMagic)
      return api_fail(TS_E_INVALID, "invalid target or transform handle");
    const bool two = x->n_inputs == 2;
    if (!ts_ok_array_handle(a) || !ts_ok_array_handle(d) || (two && !ts_ok_array_handle(b)))
      return api_fail(TS_E_INVALID, "invalid array handle");
    if (a->dtype != x->dtype) return api_fail(TS_E_DTYPE, "arrays have another storage type than the transform");
    if (x->device != t->device) return api_fail(TS_E_PLACEMENT, "transform was compiled for another device");
    const Operand ox{reinterpret_cast<uintptr_t>(a->ptr), a->n, a->dtype, a->device};
    const Operand od{reinterpret_cast<uintptr_t>(d->ptr), d->n, d->dtype, d->device};
    Operand oy{};
    if (two) oy = Operand{reinterpret_cast<uintptr_t>(b->ptr), b->n, b->dtype, b->device};
    const MapCheck c = check_map(two, t->device, ox, two ? &oy : nullptr, od);
    if (c.status != ST_OK) return api_fail(c.status, "%s", c.msg.c_str());
    if (c.count == 0) return TS_OK;
    if (t->host) {  // every worker runs the compiled function over its block
      const void* xp = a->ptr;
      const void* yp = two ? b->ptr : a->ptr;
      void* dp = d->ptr;
      const uint64_t n = c.count;
      const int W = t->pool->size();
      const HostTransformFn fn = x->host_fn;
      t->pool->run([&](int w) {
        uint64_t lo, hi;
        HostPool::block(n, W, w, &lo, &hi);
        fn(xp, yp, dp, q, lo, hi);
      });
      return TS_OK;
    }
    hipError_t he = hipSetDevice(t->device);
    if (he != hipSuccess) return api_hip_fail(he, "hipSetDevice");
    const void* xp = a->ptr;
    const void* yp = two ? b->ptr : a->ptr;
    void* dp = d->ptr;
    const unsigned long long n = c.count;
    const unsigned long long es = dtype_size(a->dtype);
    const uintptr_t xa = reinterpret_cast<uintptr_t>(xp), ya = reinterpret_cast<uintptr_t>(yp),
                    da = reinterpret_cast<uintptr_t>(dp);
    // One wave per workgroup and one vector per lane, 8 bytes when two
    // arrays are read and 16 when one is: the shapes that stream fastest at
    // sizes beyond the caches, as for the tuned maps.
    const unsigned long long vw = two ? 8 : 16;
    const unsigned long long per_vec = vw / es;
    if ((xa - da) % vw == 0 && (ya - da) % vw == 0) {
      const unsigned block = 64;
      // Shared misalignment: element-wise head up to the next vw-byte
      // boundary of every operand, vectors, element-wise tail.
      unsigned long long head = ((vw - da % vw) % vw) / es;
      if (head > n) head = n;
      const unsigned long long nvec = (n - head) / per_vec;
      const unsigned long long tail = n - head - nvec * per_vec;
      unsigned long long lanes = nvec > head ? nvec : head;
      if (tail > lanes) lanes = tail;
      // one pass of one vector per lane, capped (the kernel strides over the rest)
      const unsigned long long grid = cap_grid((lanes + block - 1) / block, block);
      void* args[] = {&xp, &yp, &dp, &q, &head, const_cast<unsigned long long*>(&nvec),
                      const_cast<unsigned long long*>(&tail)};
      he = hipModuleLaunchKernel(vw == 16 ? x->fn_vec : x->fn_vec8, static_cast<unsigned>(grid < 1 ? 1 : grid), 1,
                                 1, block, 1, 1, 0, t->stream, args, nullptr);
      if (he != hipSuccess) return api_hip_fail(he, "hipModuleLaunchKernel");
      return TS_OK;
    }
    const unsigned block = 256;
    unsigned long long nn = n;
    void* args[] = {&xp, &yp, &dp, &q, &nn};
    unsigned long long grid = (n + block - 1) / block;
    const unsigned long long cap = 32ull * static_cast<unsigned long long>(t->info.compute_units);
    if (grid > cap) grid = cap;  // grid-stride over the rest
    he = hipModuleLaunchKernel(x->fn, static_cast<unsigned>(grid), 1, 1, block, 1, 1, 0, t->stream, args, nullptr);
    if (he != hipSuccess) return api_hip_fail(he, "hipModuleLaunchKernel");
    return TS_OK;
  } catch (...) {
    return api_fail(TS_E_INVALID, "internal error");
  }
}

int ts_transform_log(ts_transform x, const char** log) {
  if (!x || x->magic != kTransformMagic || !log) return api_fail(TS_E_INVALID, "invalid transform handle");
  *log = x->log.c_str();
  return TS_OK;
}

int ts_transform_destroy(ts_transform x) {
  if (!x) return TS_OK;
  if (x->magic != kTransformMagic) return api_fail(TS_E_INVALID, "invalid transform handle");
  if (x->module) {  // host transforms keep their shared object cached for the process
    (void)hipSetDevice(x->device);
    (void)hipDeviceSynchronize();  // launches of it may still run on any stream of the device
    (void)hipModuleUnload(x->module);
  }
  x->magic = 0xdeadbeefu;
  delete x;
  return TS_OK;
}

}  // extern "C"
