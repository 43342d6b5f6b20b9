// Level application of the sparse factor and the log-determinant reduction.
//
// Forward (Alg. 1): for each batch in depth order, every point of the batch
// computes v_i = b_i . v[c(i)] + sigma_i xi_i; all its neighbours belong to
// earlier batches, so one launch per batch is race free.  Inverse (abstract,
// "inverse application"): xi_i = (v_i - b_i . v[c(i)]) / sigma_i has no
// dependency between points and runs as one launch.
//
// Both are HBM bound gather-dots: one lane per point, 64 points per wave
// reading entry m of their tiled rows as one contiguous 256-byte segment
// (neighbour index and coefficient), then gathering v.  FP32 storage uses
// FP32 accumulation.
#include "common.h"
#include "lanes.h"

namespace vk {

template <typename T, int KP, bool INVERSE>
__global__ __launch_bounds__(kBlock) void apply_kernel(const int32_t* __restrict__ nbr, const T* __restrict__ b,
                                                       const T* __restrict__ sig, const T* in, T* out, int n0,
                                                       int64_t first_tile, int64_t s_begin, int64_t s_end,
                                                       int64_t nblocks) {
    // forward: in = xi, out = v (gathered); inverse: in = v (gathered), out = xi
    const int64_t blk = xcd_block(blockIdx.x, nblocks);
    const int64_t sp = first_tile * kTile + blk * kBlock + threadIdx.x;
    if (sp < s_begin || sp >= s_end) return;
    const int64_t base = (sp >> 6) * (int64_t)KP * kTile + (sp & 63);
    const T* vsrc = INVERSE ? in : out;
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < KP; ++m) {
        const int32_t j = __builtin_nontemporal_load(nbr + base + m * kTile);
        const T w = __builtin_nontemporal_load(b + base + m * kTile);
        const T vj = vsrc[j >= 0 ? j : 0];
        acc = fma(w, j >= 0 ? vj : T(0), acc);
    }
    const int64_t s = n0 + sp;
    if constexpr (INVERSE) {
        out[s] = (in[s] - acc) / sig[sp];
    } else {
        out[s] = fma(sig[sp], in[s], acc);
    }
}

template <typename T, bool INVERSE>
static hipError_t launch_apply_t(int kp, const int32_t* nbr, const void* b, const void* sig, const void* in, void* out,
                                 int n0, int64_t s_begin, int64_t s_end, hipStream_t s) {
    if (s_end <= s_begin) return hipSuccess;
    const int64_t t0 = s_begin / kTile, t1 = (s_end + kTile - 1) / kTile;
    const int64_t nblocks = ((t1 - t0) * kTile + kBlock - 1) / kBlock;
    const T* bp = static_cast<const T*>(b);
    const T* sp = static_cast<const T*>(sig);
    const T* ip = static_cast<const T*>(in);
    T* op = static_cast<T*>(out);
    switch (kp) {
        case 8:
            hipLaunchKernelGGL((apply_kernel<T, 8, INVERSE>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, nbr, bp, sp,
                               ip, op, n0, t0, s_begin, s_end, nblocks);
            break;
        case 16:
            hipLaunchKernelGGL((apply_kernel<T, 16, INVERSE>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, nbr, bp,
                               sp, ip, op, n0, t0, s_begin, s_end, nblocks);
            break;
        case 32:
            hipLaunchKernelGGL((apply_kernel<T, 32, INVERSE>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, nbr, bp,
                               sp, ip, op, n0, t0, s_begin, s_end, nblocks);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward_level(int precision, int kp, const int32_t* nbr, const void* b, const void* sigma,
                                const void* xi, void* v, int n0, int64_t s_begin, int64_t s_end, hipStream_t s) {
    if (precision == VECCHIA_FP32)
        return launch_apply_t<float, false>(kp, nbr, b, sigma, xi, v, n0, s_begin, s_end, s);
    return launch_apply_t<double, false>(kp, nbr, b, sigma, xi, v, n0, s_begin, s_end, s);
}

hipError_t launch_inverse_sparse(int precision, int kp, const int32_t* nbr, const void* b, const void* sigma,
                                 const void* v, void* xi, int n0, int64_t ns, hipStream_t s) {
    if (precision == VECCHIA_FP32) return launch_apply_t<float, true>(kp, nbr, b, sigma, v, xi, n0, 0, ns, s);
    return launch_apply_t<double, true>(kp, nbr, b, sigma, v, xi, n0, 0, ns, s);
}

// ---- log-determinant: 2 (sum of per-block sums of log sigma + sum log L0_jj)

struct Neumaier {
    double s = 0.0, c = 0.0;
    __device__ void add(double x) {
        const double t = s + x;
        c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    __device__ void merge(const Neumaier& o) {
        add(o.s);
        c += o.c;
    }
};

constexpr int kLdThreads = 1024;

__global__ __launch_bounds__(kLdThreads) void logdet_kernel(const double* __restrict__ part, int64_t n,
                                                            const double* __restrict__ ld0, double* __restrict__ out) {
    __shared__ double S[kLdThreads], C[kLdThreads];
    Neumaier acc;
    for (int64_t i = threadIdx.x; i < n; i += kLdThreads) acc.add(part[i]);
    S[threadIdx.x] = acc.s;
    C[threadIdx.x] = acc.c;
    __syncthreads();
    for (int stride = kLdThreads / 2; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride) {
            Neumaier a{S[threadIdx.x], C[threadIdx.x]};
            a.merge(Neumaier{S[threadIdx.x + stride], C[threadIdx.x + stride]});
            S[threadIdx.x] = a.s;
            C[threadIdx.x] = a.c;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Neumaier a{S[0], C[0]};
        a.add(*ld0);
        out[0] = 2.0 * (a.s + a.c);
    }
}

hipError_t launch_logdet(const double* ldpart, int64_t nparts, const double* ld0, double* out, hipStream_t s) {
    hipLaunchKernelGGL(logdet_kernel, dim3(1), dim3(kLdThreads), 0, s, ldpart, nparts, ld0, out);
    return hipGetLastError();
}

hipError_t launch_factor_sparse_f32(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f64(const FactorLaunch& a, hipStream_t s);

hipError_t launch_factor_sparse(const FactorLaunch& a, hipStream_t s) {
    return a.precision == VECCHIA_FP32 ? launch_factor_sparse_f32(a, s) : launch_factor_sparse_f64(a, s);
}

}  // namespace vk
