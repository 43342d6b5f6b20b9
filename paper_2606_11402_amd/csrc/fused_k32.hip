// Instantiations of the fused on-the-fly forward at k padded to 32.
#include "fused_kernel.h"

namespace vk {

hipError_t launch_forward_fused_k32(const FusedLaunch& L, hipStream_t s) { return launch_forward_fused_width<32>(L, s); }

}  // namespace vk
