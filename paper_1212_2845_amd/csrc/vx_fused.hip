// Fused step kernel (placeholder: forwards to the split path).
#include "vx_device.hpp"
#include "vx_launch.hpp"

namespace vx {

template <typename T>
hipError_t launch_fused_step(const StepArgs<T> &a, hipStream_t s) {
    return launch_split_step<T>(a, s);
}

template hipError_t launch_fused_step<float>(const StepArgs<float> &, hipStream_t);
template hipError_t launch_fused_step<double>(const StepArgs<double> &, hipStream_t);

}  // namespace vx
