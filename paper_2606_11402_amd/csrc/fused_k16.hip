// Instantiations of the fused on-the-fly forward at k padded to 16.
#include "fused_kernel.h"

namespace vk {

hipError_t launch_forward_fused_k16(const FusedLaunch& L, hipStream_t s) { return launch_forward_fused_width<16>(L, s); }

}  // namespace vk
