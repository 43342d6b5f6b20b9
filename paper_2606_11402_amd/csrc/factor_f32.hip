// Instantiations of the sparse factor kernel for float storage.
#include "factor_kernel.h"

namespace vk {

template <int K>
static hipError_t dispatch_kind_f32(const FactorLaunch& a, hipStream_t s) {
    switch (a.kind) {
        case 0: return launch_factor_sparse_t<float, K, 0>(a, s);
        case 1: return launch_factor_sparse_t<float, K, 1>(a, s);
        case 2: return launch_factor_sparse_t<float, K, 2>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_factor_sparse_f32(const FactorLaunch& a, hipStream_t s) {
    switch (a.kp) {
        case 8: return dispatch_kind_f32<8>(a, s);
        case 16: return dispatch_kind_f32<16>(a, s);
        case 32: return dispatch_kind_f32<32>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace vk
