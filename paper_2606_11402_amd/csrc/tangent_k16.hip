// Instantiations of the per-point tangent of Eq. (2) at k padded to 16.
#include "tangent.h"

namespace vk {

hipError_t launch_tangent_factor_k16(const TangentLaunch& L, hipStream_t s) { return launch_tangent_factor_width<16>(L, s); }

}  // namespace vk
