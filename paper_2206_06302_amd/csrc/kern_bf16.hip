// kern_bf16.hip -- instantiation of the STREAM kernels for bf16 storage.
// One translation unit per storage format so the instances compile in
// parallel; the kernels themselves are in ts_device.hpp.
#include "ts_device.hpp"
#include "ts_internal.hpp"

namespace ts {
hipError_t plain_launch_bf16(const PlainLaunch& L) { return plain_dispatch<DT_BF16>(L); }
hipError_t batch_launch_bf16(const BatchLaunch& L) { return batch_dispatch<DT_BF16>(L); }
}  // namespace ts
