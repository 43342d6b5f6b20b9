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
// (neighbour index and coefficient), then gathering v.  The forward
// accumulates in the storage precision, the inverse in double.
#include "apply.h"
#include "lanes.h"

#include <algorithm>
#include <type_traits>

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
    // The inverse subtracts two nearly equal numbers (v_i and its conditional
    // mean) and divides by a possibly small sigma_i, so it accumulates in
    // double; double FMA runs at the FP32 rate on CDNA4 and this kernel is
    // bound by HBM, so the wider accumulator is free.  The forward sum can
    // cancel too (sum |b_m v_m| reaches ~7 max|v| on the radial Matern cloud)
    // but its result is not divided by sigma_i: with float coefficients and
    // values, float accumulation adds ~4e-7 of max|v| there (CPU emulation),
    // so it accumulates in the storage precision, as the float path specifies.
    using Acc = typename std::conditional<INVERSE, double, T>::type;
    const T* vsrc = INVERSE ? in : out;
    Acc acc = Acc(0);
#pragma unroll
    for (int m = 0; m < KP; ++m) {
        const int32_t j = __builtin_nontemporal_load(nbr + base + m * kTile);
        const T w = __builtin_nontemporal_load(b + base + m * kTile);
        const T vj = vsrc[j >= 0 ? j : 0];
        acc = fma((Acc)w, (Acc)(j >= 0 ? vj : T(0)), acc);
    }
    const int64_t s = n0 + sp;
    if constexpr (INVERSE) {
        out[s] = (T)(((Acc)in[s] - acc) / (Acc)sig[sp]);
    } else {
        out[s] = fma(sig[sp], in[s], acc);
    }
}

// A run of consecutive small batches [l_begin, l_end) in one workgroup: the
// batches are processed in order with a workgroup barrier between them, which
// replaces one launch per batch.  The values of storage positions [lo,
// run_end) live in LDS for the whole run: positions [lo, run_start) are copied
// in at the start (final values of earlier batches), the run's own outputs are
// written there as well as to v, so a gather from a batch of the run reads
// LDS after the barrier instead of making a round trip to L2; a gather below
// lo reads its (final) value from v.  A thread's first point of the next
// batch has its row (neighbour indices, coefficients, sigma, xi) loaded
// before the barrier.  The dot product runs in the same order, on the same
// values, as the per-batch kernel: the results are identical bit for bit.
template <typename T, int KP>
__global__ __launch_bounds__(run_threads(sizeof(T), KP)) void forward_run_kernel(const int32_t* __restrict__ nbr,
                                                                  const T* __restrict__ b, const T* __restrict__ sig,
                                                                  const T* __restrict__ xi, T* v, int n0,
                                                                  const int32_t* __restrict__ level_ptr, int l_begin,
                                                                  int l_end, int64_t lo) {
    constexpr int NT = run_threads(sizeof(T), KP);
    extern __shared__ unsigned char run_lds[];
    T* vl = reinterpret_cast<T*>(run_lds);             // position p at vl[p - lo]
    const int64_t run_start = level_ptr[l_begin];
    for (int64_t p = lo + threadIdx.x; p < run_start; p += NT) vl[p - lo] = v[p];
    int32_t idx[KP];
    T w[KP];
    T sg = T(0), x = T(0);
    auto load_row = [&](int64_t sp) {
        const int64_t base = (sp >> 6) * (int64_t)KP * kTile + (sp & 63);
#pragma unroll
        for (int m = 0; m < KP; ++m) {
            idx[m] = nbr[base + m * kTile];
            w[m] = b[base + m * kTile];
        }
        sg = sig[sp];
        x = xi[n0 + sp];
    };
    auto finish_row = [&](int64_t sp) {
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < KP; ++m) {
            const int32_t j = idx[m];
            // one generic (flat) load from LDS or from v, whichever holds the value
            const T* src = j >= lo ? vl + (j - lo) : v + (j >= 0 ? j : 0);
            const T vj = *src;
            acc = fma(w[m], j >= 0 ? vj : T(0), acc);
        }
        const T out = fma(sg, x, acc);
        v[n0 + sp] = out;
        vl[n0 + sp - lo] = out;
    };
    int64_t s0 = run_start - n0, s1 = (int64_t)level_ptr[l_begin + 1] - n0;
    bool have = s0 + (int64_t)threadIdx.x < s1;
    if (have) load_row(s0 + threadIdx.x);
    __syncthreads();                                   // the copied values are in LDS
    for (int l = l_begin; l < l_end; ++l) {
        if (have) finish_row(s0 + threadIdx.x);
        for (int64_t sp = s0 + threadIdx.x + NT; sp < s1; sp += NT) {
            load_row(sp);
            finish_row(sp);
        }
        int64_t t0 = s1, t1 = s1;
        if (l + 1 < l_end) {
            t0 = (int64_t)level_ptr[l + 1] - n0;
            t1 = (int64_t)level_ptr[l + 2] - n0;
        }
        have = t0 + (int64_t)threadIdx.x < t1;
        if (have) load_row(t0 + threadIdx.x);
        __syncthreads();
        s0 = t0;
        s1 = t1;
    }
}

template <typename T>
static hipError_t launch_run_t(int kp, const int32_t* nbr, const void* b, const void* sig, const void* xi, void* v,
                               int n0, const int32_t* level_ptr_dev, int l_begin, int l_end, int64_t lo,
                               int64_t run_end, hipStream_t s) {
    const T* bp = static_cast<const T*>(b);
    const T* sp = static_cast<const T*>(sig);
    const T* ip = static_cast<const T*>(xi);
    T* op = static_cast<T*>(v);
    const size_t lds = (size_t)(run_end - lo) * sizeof(T);
    if (lo < 0 || run_end < lo || lds > (size_t)kRunLdsBytes) return hipErrorInvalidValue;   // a run of empty batches has no LDS
    switch (kp) {
        case 8:
            hipLaunchKernelGGL((forward_run_kernel<T, 8>), dim3(1), dim3(run_threads(sizeof(T), 8)), lds, s, nbr,
                               bp, sp, ip, op, n0, level_ptr_dev, l_begin, l_end, lo);
            break;
        case 16:
            hipLaunchKernelGGL((forward_run_kernel<T, 16>), dim3(1), dim3(run_threads(sizeof(T), 16)), lds, s, nbr,
                               bp, sp, ip, op, n0, level_ptr_dev, l_begin, l_end, lo);
            break;
        case 32:
            hipLaunchKernelGGL((forward_run_kernel<T, 32>), dim3(1), dim3(run_threads(sizeof(T), 32)), lds, s, nbr,
                               bp, sp, ip, op, n0, level_ptr_dev, l_begin, l_end, lo);
            break;
        case 64:
            hipLaunchKernelGGL((forward_run_kernel<T, 64>), dim3(1), dim3(run_threads(sizeof(T), 64)), lds, s, nbr,
                               bp, sp, ip, op, n0, level_ptr_dev, l_begin, l_end, lo);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward_run(int precision, int kp, const int32_t* nbr, const void* b, const void* sigma,
                              const void* xi, void* v, int n0, const int32_t* level_ptr_dev, int l_begin, int l_end,
                              int64_t lo, int64_t run_end, hipStream_t s) {
    if (precision == VECCHIA_FP32)
        return launch_run_t<float>(kp, nbr, b, sigma, xi, v, n0, level_ptr_dev, l_begin, l_end, lo, run_end, s);
    return launch_run_t<double>(kp, nbr, b, sigma, xi, v, n0, level_ptr_dev, l_begin, l_end, lo, run_end, s);
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
        case 64:
            hipLaunchKernelGGL((apply_kernel<T, 64, INVERSE>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, nbr, bp,
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
constexpr int kLdBlocks = 256;   // first stage: one workgroup per CU

// Compensated sum of S[0..kLdThreads) (pairs s, c) inside one workgroup.
__device__ Neumaier block_reduce(Neumaier acc, double* S, double* C) {
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
    return Neumaier{S[0], C[0]};
}

// Stage 1: workgroup g sums a contiguous slice of the per-block partials
// (fixed slices, fixed order: the result does not depend on scheduling).
__global__ __launch_bounds__(kLdThreads) void logdet_partial_kernel(const double* __restrict__ part,
                                                                    const long long* __restrict__ fix, int64_t n,
                                                                    double* __restrict__ stage) {
    __shared__ double S[kLdThreads], C[kLdThreads];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    Neumaier acc;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kLdThreads) {
        acc.add(part[i]);
        acc.add((double)fix[i] * (1.0 / 4294967296.0));   // recomputed points of the block, 2^-32 fixed point
    }
    const Neumaier tot = block_reduce(acc, S, C);
    if (threadIdx.x == 0) {
        stage[2 * blockIdx.x] = tot.s;
        stage[2 * blockIdx.x + 1] = tot.c;
    }
}

// Stage 2: the stage-1 pairs and the dense block.
__global__ __launch_bounds__(kLdThreads) void logdet_final_kernel(const double* __restrict__ stage, int nstage,
                                                                  const double* __restrict__ ld0,
                                                                  double* __restrict__ out) {
    __shared__ double S[kLdThreads], C[kLdThreads];
    Neumaier acc;
    for (int i = threadIdx.x; i < nstage; i += kLdThreads) acc.merge(Neumaier{stage[2 * i], stage[2 * i + 1]});
    Neumaier a = block_reduce(acc, S, C);
    if (threadIdx.x == 0) {
        a.add(*ld0);
        out[0] = 2.0 * (a.s + a.c);
    }
}

__global__ void zero_u64_kernel(uint64_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_zero_u64(void* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint64_t*>(p), n);
    return hipGetLastError();
}

hipError_t launch_logdet(const double* ldpart, const long long* ldfix, int64_t nparts, const double* ld0,
                         double* stage, double* out, hipStream_t s) {
    hipLaunchKernelGGL(logdet_partial_kernel, dim3(kLdBlocks), dim3(kLdThreads), 0, s, ldpart, ldfix, nparts, stage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(logdet_final_kernel, dim3(1), dim3(kLdThreads), 0, s, stage, kLdBlocks, ld0, out);
    return hipGetLastError();
}

hipError_t launch_factor_sparse_f32_k8(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f32_k16(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f32_k32(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f64_k8(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f64_k16(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f64_k32(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f32_k64(const FactorLaunch& a, hipStream_t s);
hipError_t launch_factor_sparse_f64_k64(const FactorLaunch& a, hipStream_t s);

hipError_t launch_factor_sparse(const FactorLaunch& a, hipStream_t s) {
    const bool f32 = a.precision == VECCHIA_FP32;
    switch (a.kp) {
        case 8: return f32 ? launch_factor_sparse_f32_k8(a, s) : launch_factor_sparse_f64_k8(a, s);
        case 16: return f32 ? launch_factor_sparse_f32_k16(a, s) : launch_factor_sparse_f64_k16(a, s);
        case 32: return f32 ? launch_factor_sparse_f32_k32(a, s) : launch_factor_sparse_f64_k32(a, s);
        case 64: return f32 ? launch_factor_sparse_f32_k64(a, s) : launch_factor_sparse_f64_k64(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace vk
