// Instantiations of the sparse factor kernels: double storage, k padded to 16.
#include "factor_kernel.h"

namespace vk {

hipError_t launch_factor_sparse_f64_k16(const FactorLaunch& a, hipStream_t s) {
    switch (a.kind) {
        case 0: return launch_factor_sparse_t<double, 16, 0>(a, s);
        case 1: return launch_factor_sparse_t<double, 16, 1>(a, s);
        case 2: return launch_factor_sparse_t<double, 16, 2>(a, s);
        case 3: return launch_factor_sparse_t<double, 16, 3>(a, s);
        case 4: return launch_factor_sparse_t<double, 16, 4>(a, s);   // general Matern, FP64 only
        default: return hipErrorInvalidValue;
    }
}

}  // namespace vk
