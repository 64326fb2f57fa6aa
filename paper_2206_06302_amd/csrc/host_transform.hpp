// host_transform.hpp -- run-time compiled transforms for host-CPU targets
// (not part of the public interface).  Pure C++.
#pragma once

#include <stdint.h>

#include <string>

namespace ts {

// ds[j] = expr(xs[j], ys[j], q) for j in [lo, hi); one worker's block.
using HostTransformFn = void (*)(const void* xs, const void* ys, void* ds, double q, unsigned long long lo,
                                 unsigned long long hi);

// Compile `expr` (in x, y when n_inputs == 2, and q) for storage type
// dtype (TS_F64, TS_F32 or TS_U8) with the system C++ compiler, or return
// the cached entry point.  Returns TS_OK, TS_E_INVALID (the expression does
// not compile; *log holds the compiler's output) or TS_E_UNSUPPORTED (no
// compiler or no loader).
int host_transform_compile(const std::string& expr, int n_inputs, int dtype, HostTransformFn* fn,
                           std::string* log);

}  // namespace ts
