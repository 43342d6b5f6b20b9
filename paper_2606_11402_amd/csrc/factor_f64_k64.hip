// Instantiations of the sparse factor kernel at k padded to 64 (one point per
// wave, factor_wide.h): double storage.
#include "factor_wide.h"

namespace vk {

hipError_t launch_factor_sparse_f64_k64(const FactorLaunch& a, hipStream_t s) { return launch_factor_wide_t<double>(a, s); }

}  // namespace vk
