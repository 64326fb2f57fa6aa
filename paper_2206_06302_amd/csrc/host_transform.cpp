// host_transform.cpp -- generic transforms on host-CPU targets: the user's
// expression compiled at run time by the system C++ compiler into a small
// shared object, loaded once and run by the target's pinned workers over
// their blocks (the paper's executors run any callable on CPU and GPU alike,
// Sections 3.3 and 4.1).  Pure C++ (no HIP).
//
// The compiler is started as a child process (posix_spawnp) and the object
// is built with -ffp-contract=off -fno-fast-math, so an expression rounds
// exactly as written (fma only where the expression calls it), the same
// reading the GPU transforms use.
#include <dlfcn.h>
#include <fcntl.h>
#include <spawn.h>
#include <stdlib.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tstream.h"
#include "host_transform.hpp"

extern char** environ;

namespace ts {
namespace {

std::string host_source(const std::string& expr, int n_inputs, int dtype) {
  const char* st = dtype == TS_F64 ? "double" : dtype == TS_F32 ? "float" : "unsigned char";
  const char* at = dtype == TS_F64 ? "double" : dtype == TS_F32 ? "float" : "int";
  std::string s;
  s += "#include <cmath>\n";
  s += "using std::fma;\n";
  s += "typedef " + std::string(st) + " ts_store_t;\n";
  s += "typedef " + std::string(at) + " ts_arith_t;\n";
  s += "extern \"C\" void ts_host_transform(const void* xv, const void* yv, void* dv, double qd,\n"
       "                                    unsigned long long lo, unsigned long long hi) {\n"
       "  const ts_store_t* __restrict__ xs = static_cast<const ts_store_t*>(xv);\n"
       "  const ts_store_t* __restrict__ ys = static_cast<const ts_store_t*>(yv);\n"
       "  ts_store_t* ds = static_cast<ts_store_t*>(dv);\n"
       "  (void)ys;\n"
       "  const ts_arith_t q = (ts_arith_t)qd;\n"
       "  (void)q;\n"
       "  for (unsigned long long j = lo; j < hi; ++j) {\n"
       "    const ts_arith_t x = xs[j];\n";
  if (n_inputs == 2) s += "    const ts_arith_t y = ys[j];\n";
  s += "    ds[j] = (ts_store_t)(ts_arith_t)(" + expr + ");\n  }\n}\n";
  return s;
}

std::string read_file(const std::string& path) {
  std::ifstream f(path);
  std::stringstream ss;
  ss << f.rdbuf();
  return ss.str();
}

// Run argv as a child process with stdout and stderr sent to `log_path`;
// returns the exit status, or -errno when it could not be started.
int run_child(const std::vector<std::string>& args, const std::string& log_path) {
  std::vector<char*> argv;
  for (const std::string& a : args) argv.push_back(const_cast<char*>(a.c_str()));
  argv.push_back(nullptr);
  posix_spawn_file_actions_t fa;
  posix_spawn_file_actions_init(&fa);
  posix_spawn_file_actions_addopen(&fa, 1, log_path.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
  posix_spawn_file_actions_adddup2(&fa, 1, 2);
  pid_t pid = 0;
  const int rc = posix_spawnp(&pid, argv[0], &fa, nullptr, argv.data(), environ);
  posix_spawn_file_actions_destroy(&fa);
  if (rc != 0) return -rc;
  int status = 0;
  while (waitpid(pid, &status, 0) < 0) {
    if (errno != EINTR) return -errno;
  }
  return WIFEXITED(status) ? WEXITSTATUS(status) : 128 + (WIFSIGNALED(status) ? WTERMSIG(status) : 0);
}

std::mutex g_mu;
// Compiled entry points by (expression, inputs, storage type); the shared
// objects stay loaded for the life of the process.
std::map<std::tuple<std::string, int, int>, HostTransformFn> g_cache;

}  // namespace

int host_transform_compile(const std::string& expr, int n_inputs, int dtype, HostTransformFn* fn,
                           std::string* log) {
  std::lock_guard<std::mutex> lk(g_mu);
  const auto key = std::make_tuple(expr, n_inputs, dtype);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    *fn = it->second;
    return TS_OK;
  }
  const char* tmp = std::getenv("TMPDIR");
  std::string dir = std::string(tmp && *tmp ? tmp : "/tmp") + "/tstream-host-XXXXXX";
  if (!mkdtemp(&dir[0])) {
    *log = std::string("cannot create a build directory: ") + std::strerror(errno);
    return TS_E_UNSUPPORTED;
  }
  const std::string src = dir + "/transform.cpp", obj = dir + "/transform.so", out = dir + "/compiler.log";
  {
    std::ofstream f(src);
    f << host_source(expr, n_inputs, dtype);
  }
  const char* cxx_env = std::getenv("TS_HOST_CXX");
  const std::string cxx = cxx_env && *cxx_env ? cxx_env : "c++";
  const int rc = run_child({cxx, "-std=c++17", "-O3", "-march=native", "-fPIC", "-shared", "-ffp-contract=off",
                            "-fno-fast-math", "-o", obj, src},
                           out);
  *log = read_file(out);
  int status = TS_OK;
  if (rc < 0) {
    *log = "cannot start the host C++ compiler '" + cxx + "' (" + std::strerror(-rc) +
           "); set TS_HOST_CXX to one";
    status = TS_E_UNSUPPORTED;
  } else if (rc != 0) {
    status = TS_E_INVALID;  // the expression does not compile; the log says why
  } else {
    void* h = dlopen(obj.c_str(), RTLD_NOW | RTLD_LOCAL);
    void* sym = h ? dlsym(h, "ts_host_transform") : nullptr;
    if (!sym) {
      *log = std::string("cannot load the compiled transform: ") + dlerror();
      status = TS_E_UNSUPPORTED;
    } else {
      *fn = reinterpret_cast<HostTransformFn>(sym);
      g_cache[key] = *fn;
    }
  }
  std::remove(src.c_str());  // a loaded object may be unlinked
  std::remove(obj.c_str());
  std::remove(out.c_str());
  rmdir(dir.c_str());
  return status;
}

}  // namespace ts
