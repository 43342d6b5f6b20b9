// The theta part of the reverse-mode derivatives (adjoint.hip) for
// conditioning sets of 64 neighbours: one point per wave, lane p owns row p
// of K_cc, the factor recomputed with the left-looking Cholesky of
// factor_wide.h.  Per point (omega, sigma_bar, sbar as in adjoint.hip),
// u = K_cc^-1 bbar and
//   theta_bar += sbar dK_ii + sum_p (u_p - 2 sbar b_p) dk_p
//                + sum_{p,q} (sbar b_p - u_p) b_q dK_pq,
// lane p summing its row over q.  Double throughout; per-block partials are
// reduced in a fixed order by adj_theta_reduce_kernel.
#include "adjoint.h"
#include "factor_wide.h"

namespace vk {

template <typename TS, int KIND>
__global__ __launch_bounds__(kBlock) void adj_theta_wide_kernel(AdjArgs<TS> a) {
    __shared__ WideLds sh;
    __shared__ double red[2 * kWideWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t sp_raw = (int64_t)blockIdx.x * kWideWaves + wave;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;
    const int64_t s = a.n0 + sp;
    const double sig = (double)a.sigma[sp];
    double omega = a.vbar ? a.w[s] : 0.0;
    if (a.xibar_in) omega -= (double)a.xibar_in[s] / sig;
    const double sigma_bar = omega * (double)a.xi[s] + 2.0 * a.ldbar / sig;
    const double sbar = sigma_bar / (2.0 * sig);

    double c0, c1, c2;
    bool ok;
    wide_gather<TS>(a.x, a.nbr, sp, lane, sh.c[wave], c0, c1, c2, ok);
    const int64_t e = (sp >> 6) * (int64_t)kWide * kTile + (int64_t)lane * kTile + (sp & 63);
    const int32_t j = a.nbr[e];
    const double bq = (double)a.b[e];
    const double vj = (double)a.v[j >= 0 ? j : 0];       // unconditional load, selected below
    double u = j >= 0 ? omega * vj : 0.0;                 // bbar, then K_cc^-1 bbar

    double L[kWide];
    double inv;
    bool bad = false;
    double minpiv = 1.0;
    wide_cholesky<KIND>(sh.L[wave], sh.c[wave], c0, c1, c2, ok, lane, a.cov, a.diag, L, inv, bad, minpiv);
    (void)wide_lower_solve(L, inv, lane, u);
    wide_upper_solve(sh.L[wave], inv, lane, u);

    const TS* xt = a.x + s * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];
    const double inv_amp = 1.0 / a.sigma_amp;
    double acc_s = 0.0, acc_l = 0.0;
    {
        double kap, dl;
        cov_and_dell<KIND>(sqdist3(c0, c1, c2, t0, t1, t2), a.cov, kap, dl);
        const double coef = ok ? (u - 2.0 * sbar * bq) : 0.0;
        acc_s = fma(coef, 2.0 * kap * inv_amp, acc_s);
        acc_l = fma(coef, dl, acc_l);
    }
    const double ap = sbar * bq - u;
    static_for<0, kWide>([&](auto QI) {
        constexpr int q = QI;
        const double y0 = sh.c[wave][q][0], y1 = sh.c[wave][q][1], y2 = sh.c[wave][q][2];
        const bool okq = sh.c[wave][q][3] != 0.0;
        const double bqq = wide_readlane(bq, q);
        double kap, dl;
        cov_and_dell<KIND>(sqdist3(c0, c1, c2, y0, y1, y2), a.cov, kap, dl);
        const bool both = ok && okq;
        const bool same = lane == q;
        const double ds = both ? (same ? 2.0 * a.sigma_amp : 2.0 * kap * inv_amp) : 0.0;
        const double dll = (both && !same) ? dl : 0.0;
        acc_s = fma(ap * bqq, ds, acc_s);
        acc_l = fma(ap * bqq, dll, acc_l);
    });
    acc_s = wide_wave_sum(acc_s);
    acc_l = wide_wave_sum(acc_l);
    if (lane == 0) {
        acc_s = fma(sbar, 2.0 * a.sigma_amp, acc_s);     // dK_ii / dsigma
        red[2 * wave] = live ? acc_s : 0.0;
        red[2 * wave + 1] = live ? acc_l : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < kWideWaves; ++w) {
            s0 += red[2 * w];
            s1 += red[2 * w + 1];
        }
        a.theta_part[2 * blockIdx.x] = s0;
        a.theta_part[2 * blockIdx.x + 1] = s1;
    }
}

// Coordinates at k = 64 (the per-point terms of adj_x_kernel in adjoint.hip
// with lane p owning row p): the point's own share -sum_p k_bar_p g(x_p, x_i)
// is a wave sum; row p's share k_bar_p g(x_p, x_i) + sum_q (K_bar_pq +
// K_bar_qp) g(x_p, x_q) is summed by lane p over q and stored in the tiled
// layout for the children gather.
template <typename TS, int KIND>
__global__ __launch_bounds__(kBlock) void adj_x_wide_kernel(AdjArgs<TS> a, double* __restrict__ contrib) {
    __shared__ WideLds sh;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t sp_raw = (int64_t)blockIdx.x * kWideWaves + wave;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;
    const int64_t s = a.n0 + sp;
    const double sig = (double)a.sigma[sp];
    double omega = a.vbar ? a.w[s] : 0.0;
    if (a.xibar_in) omega -= (double)a.xibar_in[s] / sig;
    const double sigma_bar = omega * (double)a.xi[s] + 2.0 * a.ldbar / sig;
    const double sbar = sigma_bar / (2.0 * sig);

    double c0, c1, c2;
    bool ok;
    wide_gather<TS>(a.x, a.nbr, sp, lane, sh.c[wave], c0, c1, c2, ok);
    const int64_t e = (sp >> 6) * (int64_t)kWide * kTile + (int64_t)lane * kTile + (sp & 63);
    const int32_t j = a.nbr[e];
    const double bq = (double)a.b[e];
    const double vj = (double)a.v[j >= 0 ? j : 0];       // unconditional load, selected below
    double u = j >= 0 ? omega * vj : 0.0;                 // bbar, then K_cc^-1 bbar

    double L[kWide];
    double inv;
    bool bad = false;
    double minpiv = 1.0;
    wide_cholesky<KIND>(sh.L[wave], sh.c[wave], c0, c1, c2, ok, lane, a.cov, a.diag, L, inv, bad, minpiv);
    (void)wide_lower_solve(L, inv, lane, u);
    wide_upper_solve(sh.L[wave], inv, lane, u);

    const TS* xt = a.x + s * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];
    double g0, g1, g2;
    {
        double kap, ds;
        cov_and_dr<KIND>(sqdist3(c0, c1, c2, t0, t1, t2), a.cov, kap, ds);
        const double w = ok ? (u - 2.0 * sbar * bq) * ds : 0.0;
        g0 = w * (c0 - t0);
        g1 = w * (c1 - t1);
        g2 = w * (c2 - t2);
    }
    const double own0 = -wide_wave_sum(g0), own1 = -wide_wave_sum(g1), own2 = -wide_wave_sum(g2);
    static_for<0, kWide>([&](auto QI) {
        constexpr int q = QI;
        const double y0 = sh.c[wave][q][0], y1 = sh.c[wave][q][1], y2 = sh.c[wave][q][2];
        const bool okq = sh.c[wave][q][3] != 0.0;
        const double bqq = wide_readlane(bq, q), uq = wide_readlane(u, q);
        double kap, ds;
        cov_and_dr<KIND>(sqdist3(c0, c1, c2, y0, y1, y2), a.cov, kap, ds);
        const double w = (ok && okq && lane != q) ? (2.0 * sbar * bq * bqq - u * bqq - uq * bq) * ds : 0.0;
        g0 = fma(w, c0 - y0, g0);
        g1 = fma(w, c1 - y1, g1);
        g2 = fma(w, c2 - y2, g2);
    });
    if (!live) return;
    contrib[3 * e] = g0;
    contrib[3 * e + 1] = g1;
    contrib[3 * e + 2] = g2;
    if (lane == 0) {
        a.xgrad[s * 3] = own0;
        a.xgrad[s * 3 + 1] = own1;
        a.xgrad[s * 3 + 2] = own2;
    }
}

template <typename TS>
hipError_t launch_adj_x_wide(const AdjArgs<TS>& a, int kind, double* contrib, hipStream_t s) {
    switch (kind) {
        case 0: hipLaunchKernelGGL((adj_x_wide_kernel<TS, 0>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, contrib); break;
        case 1: hipLaunchKernelGGL((adj_x_wide_kernel<TS, 1>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, contrib); break;
        case 2: hipLaunchKernelGGL((adj_x_wide_kernel<TS, 2>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, contrib); break;
        case 3: hipLaunchKernelGGL((adj_x_wide_kernel<TS, 3>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a, contrib); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_adj_x_wide<float>(const AdjArgs<float>&, int, double*, hipStream_t);
template hipError_t launch_adj_x_wide<double>(const AdjArgs<double>&, int, double*, hipStream_t);

template <typename TS>
hipError_t launch_adj_theta_wide(const AdjArgs<TS>& a, int kind, hipStream_t s) {
    switch (kind) {
        case 0: hipLaunchKernelGGL((adj_theta_wide_kernel<TS, 0>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL((adj_theta_wide_kernel<TS, 1>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((adj_theta_wide_kernel<TS, 2>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((adj_theta_wide_kernel<TS, 3>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_adj_theta_wide<float>(const AdjArgs<float>&, int, hipStream_t);
template hipError_t launch_adj_theta_wide<double>(const AdjArgs<double>&, int, hipStream_t);

}  // namespace vk
