// Fused on-the-fly forward at k padded to 64: one point per wave with the
// left-looking Cholesky of factor_wide.h; w = L^-1 v[c(i)] by the same
// forward substitution as y = L^-1 k_ci, and v_i = y . w + sigma_i xi_i.
#include "factor_wide.h"
#include "fused_kernel.h"

namespace vk {

template <typename TS, int KIND>
__global__ __launch_bounds__(kBlock) void forward_fused_wide_kernel(FusedArgs<TS> a, Cov<double> cov) {
    __shared__ WideLds sh;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t blk = xcd_block(blockIdx.x, a.nblocks);
    const int64_t sp_raw = a.s_begin + blk * kWideWaves + wave;
    const bool live = sp_raw < a.s_end;
    const int64_t sp = live ? sp_raw : a.s_end - 1;
    double c0, c1, c2;
    bool ok;
    wide_gather<TS>(a.x, a.nbr, sp, lane, sh.c[wave], c0, c1, c2, ok);
    const int32_t j = a.nbr[(sp >> 6) * (int64_t)kWide * kTile + (int64_t)lane * kTile + (sp & 63)];
    const TS vj = a.v[j >= 0 ? j : 0];                       // unconditional load, selected below
    double w = j >= 0 ? (double)vj : 0.0;
    const TS* xt = a.x + (a.n0 + sp) * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];
    double L[kWide];
    double inv;
    bool bad = false;
    double minpiv = a.diag;
    wide_cholesky<KIND>(sh.L[wave], sh.c[wave], c0, c1, c2, ok, lane, cov, a.diag, L, inv, bad, minpiv);
    double y = ok ? cov_r2<KIND>(sqdist3(c0, c1, c2, t0, t1, t2), cov) : 0.0;
    const double s2 = a.diag - wide_lower_solve(L, inv, lane, y);
    (void)wide_lower_solve(L, inv, lane, w);
    const double mean = wide_wave_sum(y * w);
    bad |= !(s2 > 0.0);
    if (live && lane == 0) {
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

template <typename TS>
static hipError_t launch_wide_t(const FusedLaunch& L, hipStream_t s) {
    FusedArgs<TS> a{static_cast<const TS*>(L.x), L.nbr, static_cast<const TS*>(L.xi), static_cast<TS*>(L.v),
                    L.ldfix, L.status, L.s_begin, L.s_end, 0, L.n0, L.diag};
    a.nblocks = (a.s_end - a.s_begin + kWideWaves - 1) / kWideWaves;
    if (a.nblocks <= 0) return hipSuccess;
    const Cov<double> cov = make_cov<double>(L.kern);
    switch (L.kind) {
        case 0: hipLaunchKernelGGL((forward_fused_wide_kernel<TS, 0>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        case 1: hipLaunchKernelGGL((forward_fused_wide_kernel<TS, 1>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        case 2: hipLaunchKernelGGL((forward_fused_wide_kernel<TS, 2>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        case 3: hipLaunchKernelGGL((forward_fused_wide_kernel<TS, 3>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, cov); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward_fused_k64(const FusedLaunch& L, hipStream_t s) {
    return L.precision == VECCHIA_FP32 ? launch_wide_t<float>(L, s) : launch_wide_t<double>(L, s);
}

}  // namespace vk
