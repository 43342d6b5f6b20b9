// Fused on-the-fly forward (Alg. 1 as written): for one batch, every point
// assembles K_cc, k_ci and K_ii from the coordinates, factors K_cc, and
// produces v_i = k_ic K_cc^-1 v[c(i)] + sigma_i xi_i directly, with
// sigma_i^2 = K_ii - k_ic K_cc^-1 k_ci.  No coefficient vector is stored (the
// method's memory then scales with N, not N k), at the price of the factor's
// arithmetic in every forward pass.  Arithmetic is double for both storage
// types (the FP32 path's all-double branch); v, xi and the coordinates are
// stored in TS.  Each point adds 0.5 log sigma_i^2 to the 2^-32 fixed-point
// sum of its 64-point tile (integer atomics commute: the logdet does not
// depend on the schedule), so the pass also yields the log-determinant.
#pragma once

#include "factor_kernel.h"

namespace vk {

template <typename TS>
struct FusedArgs {
    const TS* x;           // N x 3, storage order
    const int32_t* nbr;    // tiled neighbour indices
    const TS* xi;          // N
    TS* v;                 // N: read at the neighbours (earlier batches), written at the batch's points
    long long* ldfix;      // per 64-point tile, fixed point 2^-32
    uint64_t* status;      // [first bad position, bad count, ...]
    int64_t s_begin, s_end, nblocks;   // sparse indices of the batch, workgroups of this launch
    int n0;
    double diag;           // K_ii = sigma^2 + nugget
};

template <typename TS, int K, int KIND>
__global__ __launch_bounds__(kBlock, factor_min_waves(8, K)) void forward_fused_kernel(FusedArgs<TS> a,
                                                                                         Cov<double> cov) {
    constexpr int P = factor_lanes(VECCHIA_FP64, K);
    constexpr int R = K / P;
    constexpr int PTS = kBlock / P;
    const int tid = threadIdx.x;
    const int r = tid % P;
    const int64_t blk = xcd_block(blockIdx.x, a.nblocks);
    const int64_t sp_raw = a.s_begin + blk * PTS + tid / P;
    const bool live = sp_raw < a.s_end;
    const int64_t sp = live ? sp_raw : a.s_end - 1;    // dead lanes mirror a live point
    double y[R];
    double s2, minpiv, mean = 0.0;
    bool bad;
    factor_point<double, TS, K, P, KIND, false, true, TS>(a.x, a.nbr, a.n0, sp, r, cov, a.diag, y, s2, minpiv, bad,
                                                         a.v, &mean);
    if (live && r == 0) {
        const int64_t s = a.n0 + sp;
        a.v[s] = (TS)fma(sqrt(s2), (double)a.xi[s], mean);
        if (bad) {
            atomicMin((unsigned long long*)&a.status[0], (unsigned long long)s);
            atomicAdd((unsigned long long*)&a.status[1], 1ull);
        } else {
            const long long f = __double2ll_rn(0.5 * log(s2) * kFixScale);
            atomicAdd((unsigned long long*)&a.ldfix[sp >> 6], (unsigned long long)f);
        }
    }
}

template <typename TS, int K>
hipError_t launch_forward_fused_t(int kind, const FusedArgs<TS>& args, const vecchia_kernel& kern, hipStream_t s) {
    constexpr int PTS = kBlock / factor_lanes(VECCHIA_FP64, K);
    FusedArgs<TS> a = args;
    a.nblocks = (a.s_end - a.s_begin + PTS - 1) / PTS;
    if (a.nblocks <= 0) return hipSuccess;
    const Cov<double> cov = make_cov<double>(kern);
    switch (kind) {
        case 0: hipLaunchKernelGGL((forward_fused_kernel<TS, K, 0>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        case 1: hipLaunchKernelGGL((forward_fused_kernel<TS, K, 1>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        case 2: hipLaunchKernelGGL((forward_fused_kernel<TS, K, 2>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        case 3: hipLaunchKernelGGL((forward_fused_kernel<TS, K, 3>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Launchers, one translation unit per width (the heavy templates compile in
// parallel).  precision selects TS; args are untyped here.
struct FusedLaunch {
    int precision, kp, kind, n0;
    const void* x;
    const int32_t* nbr;
    const void* xi;
    void* v;
    long long* ldfix;
    uint64_t* status;
    int64_t s_begin, s_end;
    double diag;
    vecchia_kernel kern;
};

template <int K>
hipError_t launch_forward_fused_width(const FusedLaunch& L, hipStream_t s) {
    if (L.precision == VECCHIA_FP32) {
        FusedArgs<float> a{static_cast<const float*>(L.x), L.nbr, static_cast<const float*>(L.xi),
                           static_cast<float*>(L.v), L.ldfix, L.status, L.s_begin, L.s_end, 0, L.n0, L.diag};
        return launch_forward_fused_t<float, K>(L.kind, a, L.kern, s);
    }
    FusedArgs<double> a{static_cast<const double*>(L.x), L.nbr, static_cast<const double*>(L.xi),
                        static_cast<double*>(L.v), L.ldfix, L.status, L.s_begin, L.s_end, 0, L.n0, L.diag};
    return launch_forward_fused_t<double, K>(L.kind, a, L.kern, s);
}

hipError_t launch_forward_fused_k8(const FusedLaunch& L, hipStream_t s);
hipError_t launch_forward_fused_k16(const FusedLaunch& L, hipStream_t s);
hipError_t launch_forward_fused_k32(const FusedLaunch& L, hipStream_t s);
hipError_t launch_forward_fused_k64(const FusedLaunch& L, hipStream_t s);

}  // namespace vk
