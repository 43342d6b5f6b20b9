// Dense initial batch (Sec. 2.2 "Batch construction", first line of Alg. 1):
// the first n0 values are generated jointly with the Cholesky factor of
// K[0:n0, 0:n0], always in double.  n0 <= 128, so the whole block sits in
// one workgroup's LDS (n0 x (n0+1) doubles, 132 KB of gfx950's 160 KB); the
// factor is written to the workspace as L0 (row-major, zero upper part).
#include "apply.h"

namespace vk {

constexpr int kDenseThreads = VECCHIA_N0MAX;   // one thread per row (dense forward / inverse)
constexpr int kLd = VECCHIA_N0MAX + 1;        // padded LDS row stride
constexpr int kDenseCols = 8;                 // factor: threads per row, each on every 8th column
constexpr int kDenseFactorThreads = VECCHIA_N0MAX * kDenseCols;

// Right-looking Cholesky in LDS.  Thread (i, c) owns the columns c, c + 8,
// ... of row i, so the rank-1 update of step j spreads row i's (i - j)
// entries over 8 threads; every entry still receives its updates one step
// after the other, in the same order as with one thread per row.
template <typename TX, int KIND>
__global__ __launch_bounds__(kDenseFactorThreads) void factor_dense_kernel(const TX* __restrict__ x, int n0,
                                                                             Cov<double> cov, double nugget,
                                                                             double* __restrict__ l0,
                                                                             double* __restrict__ ld0,
                                                                             uint64_t* __restrict__ status) {
    __shared__ double A[VECCHIA_N0MAX * kLd];
    const int tid = threadIdx.x;
    const int i = tid / kDenseCols, c = tid % kDenseCols;
    if (tid == 0) {
        status[0] = kStatusNone;   // first failing storage position
        status[1] = 0;             // failing points
        status[2] = 0;             // FP32 path: points recomputed in double
        status[3] = 0;             // unused
        status[4] = 0;             // unused
        status[5] = 0;             // FP32 policy sample: points that would be recomputed in double
        status[6] = 0;             // FP32 policy sample: points looked at
    }
    if (i < n0) {
        const double a0 = (double)x[i * 3 + 0], a1 = (double)x[i * 3 + 1], a2 = (double)x[i * 3 + 2];
        for (int l = c; l <= i; l += kDenseCols) {
            const double r2 = sqdist3(a0, a1, a2, (double)x[l * 3 + 0], (double)x[l * 3 + 1], (double)x[l * 3 + 2]);
            A[i * kLd + l] = cov_r2<KIND>(r2, cov) + (l == i ? nugget : 0.0);
        }
    }
    __syncthreads();
    double lsum = 0.0;
    int bad_row = -1;
    for (int j = 0; j < n0; ++j) {
        const double d = A[j * kLd + j];
        const double sq = sqrt(d);
        if (!(d > 0.0) && bad_row < 0) bad_row = j;
        lsum += log(sq);
        __syncthreads();
        if (c == 0) {
            if (i == j) A[j * kLd + j] = sq;
            if (i > j && i < n0) A[i * kLd + j] = A[i * kLd + j] / sq;
        }
        __syncthreads();
        if (i > j && i < n0) {
            const double lij = A[i * kLd + j];
            for (int l = j + 1 + c; l <= i; l += kDenseCols) A[i * kLd + l] = fma(-lij, A[l * kLd + j], A[i * kLd + l]);
        }
        __syncthreads();
    }
    if (i < n0)
        for (int l = c; l < n0; l += kDenseCols) l0[i * n0 + l] = l <= i ? A[i * kLd + l] : 0.0;
    if (tid == 0) {
        *ld0 = lsum;
        if (bad_row >= 0) {
            status[0] = (uint64_t)bad_row;
            status[1] = 1;
        }
    }
}

// v[0:n0] = L0 xi[0:n0]
template <typename T>
__global__ __launch_bounds__(kDenseThreads) void forward_dense_kernel(const double* __restrict__ l0, int n0,
                                                                       const T* __restrict__ xi, T* __restrict__ v) {
    __shared__ double z[VECCHIA_N0MAX];
    const int i = threadIdx.x;
    if (i < n0) z[i] = (double)xi[i];
    __syncthreads();
    if (i < n0) {
        double acc = 0.0;
        for (int l = 0; l <= i; ++l) acc = fma(l0[i * n0 + l], z[l], acc);
        v[i] = (T)acc;
    }
}

// xi[0:n0] = L0^-1 v[0:n0] by forward substitution, one row per thread.
template <typename T>
__global__ __launch_bounds__(kDenseThreads) void inverse_dense_kernel(const double* __restrict__ l0, int n0,
                                                                       const T* __restrict__ v, T* __restrict__ xi) {
    __shared__ double z[VECCHIA_N0MAX];
    const int i = threadIdx.x;
    double ri = i < n0 ? (double)v[i] : 0.0;
    for (int j = 0; j < n0; ++j) {
        if (i == j) z[j] = ri / l0[j * n0 + j];
        __syncthreads();
        if (i > j && i < n0) ri = fma(-l0[i * n0 + j], z[j], ri);
    }
    if (i < n0) xi[i] = (T)z[i];
}

template <typename TX>
static hipError_t launch_factor_dense_t(int kind, const void* x, int n0, const vecchia_kernel& kern, double* l0,
                                        double* ld0, uint64_t* status, hipStream_t s) {
    const Cov<double> cov = make_cov<double>(kern);
    const TX* xp = static_cast<const TX*>(x);
    switch (kind) {
        case 0:
            hipLaunchKernelGGL((factor_dense_kernel<TX, 0>), dim3(1), dim3(kDenseFactorThreads), 0, s, xp, n0, cov,
                               kern.nugget, l0, ld0, status);
            break;
        case 1:
            hipLaunchKernelGGL((factor_dense_kernel<TX, 1>), dim3(1), dim3(kDenseFactorThreads), 0, s, xp, n0, cov,
                               kern.nugget, l0, ld0, status);
            break;
        case 2:
            hipLaunchKernelGGL((factor_dense_kernel<TX, 2>), dim3(1), dim3(kDenseFactorThreads), 0, s, xp, n0, cov,
                               kern.nugget, l0, ld0, status);
            break;
        case 3:
            hipLaunchKernelGGL((factor_dense_kernel<TX, 3>), dim3(1), dim3(kDenseFactorThreads), 0, s, xp, n0, cov,
                               kern.nugget, l0, ld0, status);
            break;
        case 4:
            hipLaunchKernelGGL((factor_dense_kernel<TX, 4>), dim3(1), dim3(kDenseFactorThreads), 0, s, xp, n0, cov,
                               kern.nugget, l0, ld0, status);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_factor_dense(int precision, int kind, const void* x, int n0, const vecchia_kernel& kern, double* l0,
                               double* ld0, uint64_t* status, hipStream_t s) {
    if (precision == VECCHIA_FP32) return launch_factor_dense_t<float>(kind, x, n0, kern, l0, ld0, status, s);
    return launch_factor_dense_t<double>(kind, x, n0, kern, l0, ld0, status, s);
}

hipError_t launch_forward_dense(int precision, const double* l0, int n0, const void* xi, void* v, hipStream_t s) {
    if (precision == VECCHIA_FP32)
        hipLaunchKernelGGL(forward_dense_kernel<float>, dim3(1), dim3(kDenseThreads), 0, s, l0, n0,
                           static_cast<const float*>(xi), static_cast<float*>(v));
    else
        hipLaunchKernelGGL(forward_dense_kernel<double>, dim3(1), dim3(kDenseThreads), 0, s, l0, n0,
                           static_cast<const double*>(xi), static_cast<double*>(v));
    return hipGetLastError();
}

hipError_t launch_inverse_dense(int precision, const double* l0, int n0, const void* v, void* xi, hipStream_t s) {
    if (precision == VECCHIA_FP32)
        hipLaunchKernelGGL(inverse_dense_kernel<float>, dim3(1), dim3(kDenseThreads), 0, s, l0, n0,
                           static_cast<const float*>(v), static_cast<float*>(xi));
    else
        hipLaunchKernelGGL(inverse_dense_kernel<double>, dim3(1), dim3(kDenseThreads), 0, s, l0, n0,
                           static_cast<const double*>(v), static_cast<double*>(xi));
    return hipGetLastError();
}

}  // namespace vk
