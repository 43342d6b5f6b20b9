// Reverse-mode derivatives: arguments shared by the kernels of adjoint.hip
// and of the wide (k = 64) theta kernel in adjoint_wide.hip.
#pragma once

#include <algorithm>

#include "factor_kernel.h"

namespace vk {

// kappa(r) and d kappa / d ell (no nugget), double.
template <int KIND>
__device__ __forceinline__ void cov_and_dell(double r2, const Cov<double>& c, double& kap, double& dell) {
    if constexpr (KIND == 0) {
        const double r = sqrt(r2);
        kap = c.s2 * exp(-r * c.inv_ell);
        dell = kap * r * c.inv_ell * c.inv_ell;
    } else if constexpr (KIND == 1) {
        const double a = sqrt(r2) * c.c_m32;
        const double e = exp(-a);
        kap = c.s2 * (1.0 + a) * e;
        dell = c.s2 * a * a * e * c.inv_ell;
    } else if constexpr (KIND == 3) {
        const double a = sqrt(r2) * c.c_m52;
        const double e = exp(-a);
        kap = c.s2 * fma(a, fma(a, 1.0 / 3.0, 1.0), 1.0) * e;
        dell = c.s2 * a * a * (1.0 + a) * e * c.inv_ell * (1.0 / 3.0);
    } else {
        kap = c.s2 * exp(r2 * c.c_se);
        dell = kap * r2 * c.inv_ell * c.inv_ell * c.inv_ell;
    }
}

template <typename TS>
struct AdjArgs {
    const TS* x;
    const int32_t* nbr;
    const int64_t* child_ptr;
    const int32_t* child;
    const TS* b;
    const TS* sigma;
    const double* l0;
    const TS* xi;           // the pair (xi, v)
    const TS* v;
    const TS* vbar;         // may be null
    const TS* xibar_in;     // may be null
    double* w;              // scratch, N: the reverse sweep, double in both precisions
    TS* xibar;              // output (forward part)
    TS* vbar_out;           // output (inverse part)
    double* t0;             // scratch, n0: L0^-T xibar0
    double* theta_part;     // scratch, 2 per block of the theta kernel
    double* theta_dense;    // scratch, 2
    double* theta_out;      // output, 2
    int64_t n, ns, nblocks;
    int n0, kp;
    double ldbar;
    double sigma_amp;
    double diag;            // K_ii = sigma^2 + nugget
    Cov<double> cov;
    double* xgrad = nullptr;  // coordinate cotangents (N x 3, storage order), or null: theta only
};

// kappa(r) and kappa'(r) / r (no nugget), double; the latter is the factor of
// (x_p - x_q) in d kappa(|x_p - x_q|) / d x_p, zero where the points coincide.
template <int KIND>
__device__ __forceinline__ void cov_and_dr(double r2, const Cov<double>& c, double& kap, double& dscale) {
    if constexpr (KIND == 0) {
        const double r = sqrt(r2);
        kap = c.s2 * exp(-r * c.inv_ell);
        dscale = r > 0.0 ? -kap * c.inv_ell / r : 0.0;
    } else if constexpr (KIND == 1) {
        const double a = sqrt(r2) * c.c_m32;
        const double e = exp(-a);
        kap = c.s2 * (1.0 + a) * e;
        dscale = -c.s2 * e * c.c_m32 * c.c_m32;
    } else if constexpr (KIND == 3) {
        const double a = sqrt(r2) * c.c_m52;
        const double e = exp(-a);
        kap = c.s2 * fma(a, fma(a, 1.0 / 3.0, 1.0), 1.0) * e;
        dscale = -c.s2 * (1.0 + a) * e * c.c_m52 * c.c_m52 * (1.0 / 3.0);
    } else {
        kap = c.s2 * exp(r2 * c.c_se);
        dscale = 2.0 * c.c_se * kap;
    }
}

__device__ __forceinline__ void block_sum2(double& s0, double& s1, double* sh) {
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
    }
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[2 * wv] = s0;
        sh[2 * wv + 1] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = 0.0, a1 = 0.0;
        for (int w = 0; w < nw; ++w) {
            a0 += sh[2 * w];
            a1 += sh[2 * w + 1];
        }
        s0 = a0;
        s1 = a1;
    }
}

template <typename TS>
hipError_t launch_adj_theta_wide(const AdjArgs<TS>& a, int kind, hipStream_t s);
template <typename TS>
hipError_t launch_adj_x_wide(const AdjArgs<TS>& a, int kind, double* contrib, hipStream_t s);

}  // namespace vk
