// Instantiations of the fused on-the-fly forward at k padded to 8.
#include "fused_kernel.h"

namespace vk {

hipError_t launch_forward_fused_k8(const FusedLaunch& L, hipStream_t s) { return launch_forward_fused_width<8>(L, s); }

}  // namespace vk
