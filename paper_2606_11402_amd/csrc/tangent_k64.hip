// The per-point tangent of Eq. (2) (tangent.h) at k padded to 64: one point
// per wave, lane p owns row p, K_cc factored by the left-looking Cholesky of
// factor_wide.h.
#include "factor_wide.h"
#include "tangent.h"

namespace vk {

template <typename TS, int KIND>
__global__ __launch_bounds__(kBlock) void tangent_factor_wide_kernel(TangentArgs<TS> a) {
    __shared__ WideLds sh;
    __shared__ double red[kWideWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t blk = xcd_block(blockIdx.x, a.nblocks);
    const int64_t sp_raw = blk * kWideWaves + wave;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;
    double c0, c1, c2;
    bool ok;
    wide_gather<TS>(a.x, a.nbr, sp, lane, sh.c[wave], c0, c1, c2, ok);
    const int64_t e = (sp >> 6) * (int64_t)kWide * kTile + (int64_t)lane * kTile + (sp & 63);
    const double bq = ok ? (double)a.b[e] : 0.0;
    const TS* xt = a.x + (a.n0 + sp) * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];
    double u = ok ? kappa_dot<KIND>(sqdist3(c0, c1, c2, t0, t1, t2), a.cov, a.sigma_amp, a.sdot, a.ldot) : 0.0;
    const double kcb = wide_wave_sum(u * bq);
    double kdb = 0.0;
    static_for<0, kWide>([&](auto QI) {
        constexpr int q = QI;
        const double y0 = sh.c[wave][q][0], y1 = sh.c[wave][q][1], y2 = sh.c[wave][q][2];
        const double bqq = wide_readlane(bq, q);
        kdb = fma(kappa_dot<KIND>(sqdist3(c0, c1, c2, y0, y1, y2), a.cov, a.sigma_amp, a.sdot, a.ldot), bqq, kdb);
    });
    u = ok ? u - kdb : 0.0;
    const double bkb = wide_wave_sum(bq * kdb);
    double L[kWide];
    double inv;
    bool bad = false;
    double minpiv = a.diag;
    wide_cholesky<KIND>(sh.L[wave], sh.c[wave], c0, c1, c2, ok, lane, a.cov, a.diag, L, inv, bad, minpiv);
    (void)wide_lower_solve(L, inv, lane, u);
    wide_upper_solve(sh.L[wave], inv, lane, u);
    const double sig = (double)a.sigma[sp];
    const double sdot = (a.sdot * 2.0 * a.sigma_amp - 2.0 * kcb + bkb) / (2.0 * sig);
    if (live) {
        a.bdot[e] = (TS)u;
        if (lane == 0) a.sigdot[sp] = (TS)sdot;
    }
    if (lane == 0) red[wave] = live ? sdot / sig : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kWideWaves; ++w) s += red[w];
        a.part[blk] = s;
    }
}

template <typename TS>
static hipError_t launch_wide_t(const TangentLaunch& L, hipStream_t s) {
    TangentArgs<TS> a{static_cast<const TS*>(L.x), L.nbr, static_cast<const TS*>(L.b),
                      static_cast<const TS*>(L.sigma), static_cast<TS*>(L.bdot), static_cast<TS*>(L.sigdot), L.part,
                      L.ns, 0, L.n0, L.diag, L.sigma_amp, L.sdot, L.ldot, make_cov<double>(L.kern)};
    a.nblocks = (a.ns + kWideWaves - 1) / kWideWaves;
    if (a.nblocks == 0) return hipSuccess;
    switch (L.kind) {
        case 0: hipLaunchKernelGGL((tangent_factor_wide_kernel<TS, 0>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL((tangent_factor_wide_kernel<TS, 1>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((tangent_factor_wide_kernel<TS, 2>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((tangent_factor_wide_kernel<TS, 3>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tangent_factor_k64(const TangentLaunch& L, hipStream_t s) {
    return L.precision == VECCHIA_FP32 ? launch_wide_t<float>(L, s) : launch_wide_t<double>(L, s);
}

}  // namespace vk
