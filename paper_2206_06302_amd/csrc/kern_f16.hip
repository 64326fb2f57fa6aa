// kern_f16.hip -- instantiation of the STREAM kernels for f16 storage.
// One translation unit per storage format so the instances compile in
// parallel; the kernels themselves are in ts_device.hpp.
#include "ts_device.hpp"
#include "ts_internal.hpp"

namespace ts {
hipError_t plain_launch_f16(const PlainLaunch& L) { return plain_dispatch<DT_F16>(L); }
hipError_t batch_launch_f16(const BatchLaunch& L) { return batch_dispatch<DT_F16>(L); }
}  // namespace ts
