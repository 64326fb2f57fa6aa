// kern_f32.hip -- instantiation of the STREAM kernels for f32 storage.
// One translation unit per storage format so the instances compile in
// parallel; the kernels themselves are in ts_device.hpp.
#include "ts_device.hpp"
#include "ts_internal.hpp"

namespace ts {
hipError_t plain_launch_f32(const PlainLaunch& L) { return plain_dispatch<DT_F32>(L); }
hipError_t batch_launch_f32(const BatchLaunch& L) { return batch_dispatch<DT_F32>(L); }
}  // namespace ts
