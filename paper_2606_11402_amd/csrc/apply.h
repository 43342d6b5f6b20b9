// Level application of the sparse factor (forward v = F(xi), inverse
// xi = F^-1(v)) and its dense first block: launch entry points and the
// parameters of the small-batch runs.  Kept apart from common.h so that the
// factor kernels' sources do not depend on them.
#pragma once

#include "common.h"

namespace vk {

hipError_t launch_forward_dense(int precision, const double* l0, int n0, const void* xi, void* v, hipStream_t stream);
hipError_t launch_forward_level(int precision, int kp, const int32_t* nbr, const void* b, const void* sigma,
                                const void* xi, void* v, int n0, int64_t s_begin, int64_t s_end, hipStream_t stream);
constexpr int kRunThreads = 1024;        // workgroup of the small-batch runs
// FP64 rows at k = 32 need more than the 128 registers per lane of 16 waves
// per CU; rows of 64 entries more than the 256 of 8 waves
__host__ __device__ constexpr int run_threads(int elem_bytes, int kp) {
    return kp == 64 ? kRunThreads / 4 : (elem_bytes == 8 && kp == 32 ? kRunThreads / 2 : kRunThreads);
}
constexpr int64_t kRunMaxPoints = 512;   // a batch this small joins a run
constexpr int64_t kRunLdsBytes = 65536;  // LDS copy of the positions [lo, run_end) a run reads and writes
// One workgroup over batches [l_begin, l_end); LDS holds positions [lo, run_end)
// (lo = 0 or the run's first position, (run_end - lo) * element size <= kRunLdsBytes).
hipError_t launch_forward_run(int precision, int kp, const int32_t* nbr, const void* b, const void* sigma,
                              const void* xi, void* v, int n0, const int32_t* level_ptr_dev, int l_begin, int l_end,
                              int64_t lo, int64_t run_end, hipStream_t stream);
hipError_t launch_inverse_dense(int precision, const double* l0, int n0, const void* v, void* xi, hipStream_t stream);
hipError_t launch_inverse_sparse(int precision, int kp, const int32_t* nbr, const void* b, const void* sigma,
                                 const void* v, void* xi, int n0, int64_t ns, hipStream_t stream);

}  // namespace vk
