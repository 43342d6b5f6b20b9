// Instantiations of the per-point tangent of Eq. (2) at k padded to 8.
#include "tangent.h"

namespace vk {

hipError_t launch_tangent_factor_k8(const TangentLaunch& L, hipStream_t s) { return launch_tangent_factor_width<8>(L, s); }

}  // namespace vk
