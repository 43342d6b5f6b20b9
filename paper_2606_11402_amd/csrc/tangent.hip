// The tangent pass of vecchia_forward_jvp (tangent.h): per-point tangents of
// the factor, the dense block's tangent, then the batches in order.
#include "apply.h"
#include "tangent.h"

namespace vk {

// v_dot_i = b_dot . v[c(i)] + b . v_dot[c(i)] + sigma_dot_i xi_i + sigma_i xi_dot_i
// for the points of one batch; one lane per point, double accumulation.
template <typename T, int KP>
__global__ __launch_bounds__(kBlock) void tangent_apply_kernel(const int32_t* __restrict__ nbr,
                                                               const T* __restrict__ b, const T* __restrict__ bdot,
                                                               const T* __restrict__ sig,
                                                               const T* __restrict__ sigdot,
                                                               const T* __restrict__ xi, const T* __restrict__ xidot,
                                                               const T* __restrict__ v, T* vdot, int n0,
                                                               int64_t first_tile, int64_t s_begin, int64_t s_end,
                                                               int64_t nblocks) {
    const int64_t blk = xcd_block(blockIdx.x, nblocks);
    const int64_t sp = first_tile * kTile + blk * kBlock + threadIdx.x;
    if (sp < s_begin || sp >= s_end) return;
    const int64_t base = (sp >> 6) * (int64_t)KP * kTile + (sp & 63);
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < KP; ++m) {
        const int32_t j = nbr[base + m * kTile];
        const int64_t jj = j >= 0 ? j : 0;
        const double w = (double)b[base + m * kTile], wd = (double)bdot[base + m * kTile];
        const double vj = j >= 0 ? (double)v[jj] : 0.0, vdj = j >= 0 ? (double)vdot[jj] : 0.0;
        acc = fma(wd, vj, fma(w, vdj, acc));
    }
    const int64_t s = n0 + sp;
    acc = fma((double)sigdot[sp], (double)xi[s], acc);
    if (xidot) acc = fma((double)sig[sp], (double)xidot[s], acc);
    vdot[s] = (T)acc;
}

// Dense block, one workgroup, thread i owns row i:  X = K0_dot (in LDS),
// X <- L0^-1 X (thread j solves column j), X <- X L0^-T (thread i solves row
// i), t = Phi(X) xi0 + xi0_dot, v0_dot = L0 t, ld0dot = tr(X) / 2 (the logdet
// reduction doubles it).
template <typename TS, int KIND>
__global__ __launch_bounds__(VECCHIA_N0MAX) void tangent_dense_kernel(const TS* __restrict__ x,
                                                                      const double* __restrict__ l0, int n0,
                                                                      Cov<double> cov, double sigma_amp, double sdot,
                                                                      double ldot, const TS* __restrict__ xi,
                                                                      const TS* __restrict__ xidot, TS* vdot,
                                                                      double* ld0dot) {
    constexpr int LD = VECCHIA_N0MAX + 1;
    __shared__ double X[VECCHIA_N0MAX * LD];
    __shared__ double t[VECCHIA_N0MAX];
    __shared__ double red[VECCHIA_N0MAX / 64];
    const int i = threadIdx.x;
    if (i < n0) {
        const double p0 = (double)x[i * 3], p1 = (double)x[i * 3 + 1], p2 = (double)x[i * 3 + 2];
        for (int j = 0; j < n0; ++j)
            X[i * LD + j] = kappa_dot<KIND>(sqdist3(p0, p1, p2, (double)x[j * 3], (double)x[j * 3 + 1],
                                                    (double)x[j * 3 + 2]),
                                            cov, sigma_amp, sdot, ldot);
    }
    __syncthreads();
    if (i < n0) {                                        // column i: L0 y = X[:, i]
        for (int r = 0; r < n0; ++r) {
            double m = X[r * LD + i];
            for (int l = 0; l < r; ++l) m = fma(-l0[r * n0 + l], X[l * LD + i], m);
            X[r * LD + i] = m / l0[r * n0 + r];
        }
    }
    __syncthreads();
    if (i < n0) {                                        // row i: z L0^T = X[i, :]  <=>  L0 z^T = X[i, :]^T
        for (int c = 0; c < n0; ++c) {
            double m = X[i * LD + c];
            for (int l = 0; l < c; ++l) m = fma(-l0[c * n0 + l], X[i * LD + l], m);
            X[i * LD + c] = m / l0[c * n0 + c];
        }
        double ti = 0.5 * X[i * LD + i] * (double)xi[i];
        for (int j = 0; j < i; ++j) ti = fma(X[i * LD + j], (double)xi[j], ti);
        if (xidot) ti += (double)xidot[i];
        t[i] = ti;
    }
    __syncthreads();
    double tr = 0.0;
    if (i < n0) {
        double acc = 0.0;
        for (int j = 0; j <= i; ++j) acc = fma(l0[i * n0 + j], t[j], acc);
        vdot[i] = (TS)acc;
        tr = X[i * LD + i];
    }
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
    if ((i & 63) == 0) red[i >> 6] = tr;
    __syncthreads();
    if (i == 0) {
        double s = 0.0;
        for (int w = 0; w < VECCHIA_N0MAX / 64; ++w) s += red[w];
        *ld0dot = 0.5 * s;
    }
}

template <typename T>
static hipError_t tangent_levels(const TangentLaunch& L, hipStream_t s) {
    const T* b = static_cast<const T*>(L.b);
    const T* bd = static_cast<const T*>(L.bdot);
    const T* sg = static_cast<const T*>(L.sigma);
    const T* sd = static_cast<const T*>(L.sigdot);
    const T* xi = static_cast<const T*>(L.xi);
    const T* xd = static_cast<const T*>(L.xi_dot);
    const T* v = static_cast<const T*>(L.v);
    T* vd = static_cast<T*>(L.v_dot);
    for (int l = 1; l <= L.n_levels; ++l) {
        const int64_t s_begin = L.level_ptr[l] - L.n0, s_end = L.level_ptr[l + 1] - L.n0;
        if (s_end <= s_begin) continue;
        const int64_t t0 = s_begin / kTile, t1 = (s_end + kTile - 1) / kTile;
        const int64_t nblocks = ((t1 - t0) * kTile + kBlock - 1) / kBlock;
        switch (L.kp) {
            case 8: hipLaunchKernelGGL((tangent_apply_kernel<T, 8>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, L.nbr, b, bd, sg, sd, xi, xd, v, vd, L.n0, t0, s_begin, s_end, nblocks); break;
            case 16: hipLaunchKernelGGL((tangent_apply_kernel<T, 16>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, L.nbr, b, bd, sg, sd, xi, xd, v, vd, L.n0, t0, s_begin, s_end, nblocks); break;
            case 32: hipLaunchKernelGGL((tangent_apply_kernel<T, 32>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, L.nbr, b, bd, sg, sd, xi, xd, v, vd, L.n0, t0, s_begin, s_end, nblocks); break;
            case 64: hipLaunchKernelGGL((tangent_apply_kernel<T, 64>), dim3((unsigned)nblocks), dim3(kBlock), 0, s, L.nbr, b, bd, sg, sd, xi, xd, v, vd, L.n0, t0, s_begin, s_end, nblocks); break;
            default: return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TS>
static hipError_t tangent_dense(const TangentLaunch& L, hipStream_t s) {
    const Cov<double> cov = make_cov<double>(L.kern);
    const TS* x = static_cast<const TS*>(L.x);
    const TS* xi = static_cast<const TS*>(L.xi);
    const TS* xd = static_cast<const TS*>(L.xi_dot);
    TS* vd = static_cast<TS*>(L.v_dot);
    switch (L.kind) {
        case 0: hipLaunchKernelGGL((tangent_dense_kernel<TS, 0>), dim3(1), dim3(VECCHIA_N0MAX), 0, s, x, L.l0, L.n0, cov, L.sigma_amp, L.sdot, L.ldot, xi, xd, vd, L.ld0dot); break;
        case 1: hipLaunchKernelGGL((tangent_dense_kernel<TS, 1>), dim3(1), dim3(VECCHIA_N0MAX), 0, s, x, L.l0, L.n0, cov, L.sigma_amp, L.sdot, L.ldot, xi, xd, vd, L.ld0dot); break;
        case 2: hipLaunchKernelGGL((tangent_dense_kernel<TS, 2>), dim3(1), dim3(VECCHIA_N0MAX), 0, s, x, L.l0, L.n0, cov, L.sigma_amp, L.sdot, L.ldot, xi, xd, vd, L.ld0dot); break;
        case 3: hipLaunchKernelGGL((tangent_dense_kernel<TS, 3>), dim3(1), dim3(VECCHIA_N0MAX), 0, s, x, L.l0, L.n0, cov, L.sigma_amp, L.sdot, L.ldot, xi, xd, vd, L.ld0dot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward_tangent(const TangentLaunch& L, hipStream_t s) {
    const int64_t nb = L.ns > 0 ? (L.ns + kBlock / factor_lanes(VECCHIA_FP64, L.kp) - 1) /
                                      (kBlock / factor_lanes(VECCHIA_FP64, L.kp))
                                : 0;
    hipError_t e = launch_zero_u64(L.fixzero, nb > 0 ? nb : 1, s);
    if (e != hipSuccess) return e;
    if (L.ns > 0) {
        switch (L.kp) {
            case 8: e = launch_tangent_factor_k8(L, s); break;
            case 16: e = launch_tangent_factor_k16(L, s); break;
            case 32: e = launch_tangent_factor_k32(L, s); break;
            case 64: e = launch_tangent_factor_k64(L, s); break;
            default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    e = L.precision == VECCHIA_FP32 ? tangent_dense<float>(L, s) : tangent_dense<double>(L, s);
    if (e != hipSuccess) return e;
    e = L.precision == VECCHIA_FP32 ? tangent_levels<float>(L, s) : tangent_levels<double>(L, s);
    if (e != hipSuccess) return e;
    if (L.logdet_dot)
        e = launch_logdet(L.part, reinterpret_cast<const long long*>(L.fixzero), nb, L.ld0dot, L.stage, L.logdet_dot,
                          s);
    return e;
}

}  // namespace vk
