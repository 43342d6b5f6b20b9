// Forward-mode derivatives (tangents) of forward and logdet with respect to
// xi and theta = (sigma, ell) in a direction (xi_dot, theta_dot).
//
// Differentiating Eq. (2) per sparse point (K_dot = sum_t theta_dot_t
// dK/dtheta_t, nugget excluded; b and sigma from the stored factor):
//     b_dot     = K_cc^-1 (k_dot_ci - K_dot_cc b)
//     sigma_dot = (K_dot_ii - 2 k_dot_ci . b + b . K_dot_cc b) / (2 sigma)
// and Alg. 1's recursion, batch by batch:
//     v_dot_i = b_dot . v[c(i)] + b . v_dot[c(i)] + sigma_dot_i xi_i + sigma_i xi_dot_i.
// The dense block: L0_dot = L0 Phi(X), X = L0^-1 K0_dot L0^-T (Phi: lower
// triangle, diagonal halved), v0_dot = L0 (Phi(X) xi0 + xi0_dot).  The logdet
// tangent is 2 sum sigma_dot_i / sigma_i + tr(X).  K_cc is recomputed per
// point (nothing of size k^2 stored); arithmetic is double.
#pragma once

#include "adjoint.h"

namespace vk {

template <typename TS>
struct TangentArgs {
    const TS* x;
    const int32_t* nbr;
    const TS* b;          // stored coefficients (tiled, device row order)
    const TS* sigma;
    TS* bdot;             // out: tiled like b
    TS* sigdot;           // out: per sparse point
    double* part;         // out: per block sum of sigma_dot / sigma
    int64_t ns, nblocks;
    int n0;
    double diag, sigma_amp, sdot, ldot;   // K_ii, sigma, the direction (sigma_dot, ell_dot)
    Cov<double> cov;
};

template <int KIND>
__device__ __forceinline__ double kappa_dot(double r2, const Cov<double>& c, double sigma_amp, double sdot,
                                            double ldot) {
    double kap, dl;
    cov_and_dell<KIND>(r2, c, kap, dl);
    return sdot * 2.0 * kap / sigma_amp + ldot * dl;
}

// One group of P lanes per sparse point (the layout of factor_kernel.h).
template <typename TS, int K, int KIND>
__global__ __launch_bounds__(kBlock, factor_min_waves(8, K)) void tangent_factor_kernel(TangentArgs<TS> a) {
    constexpr int P = factor_lanes(VECCHIA_FP64, K);
    constexpr int R = K / P;
    constexpr int NA = P * R * (R + 1) / 2;
    constexpr int PTS = kBlock / P;
    const int tid = threadIdx.x;
    const int r = tid % P;
    const int64_t blk = xcd_block(blockIdx.x, a.nblocks);
    const int64_t sp_raw = blk * PTS + tid / P;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;
    const int64_t base = (sp >> 6) * (int64_t)K * kTile + (sp & 63);
    const TS* xt = a.x + (int64_t)(a.n0 + sp) * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];

    double c0[R], c1[R], c2[R], bq[R];
    int ok[R];
    gather_rows<double, TS, K, P>(a.x, a.nbr, base, r, c0, c1, c2, ok);
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        bq[p] = ok[p] ? (double)a.b[base + (int64_t)(p * P + r) * kTile] : 0.0;
    });
    // u = k_dot_ci - K_dot_cc b and kb = (K_dot_cc b)_p for the rows of this lane
    double u[R], kdb[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        u[p] = ok[p] ? kappa_dot<KIND>(sqdist3(c0[p], c1[p], c2[p], t0, t1, t2), a.cov, a.sigma_amp, a.sdot, a.ldot)
                     : 0.0;
        kdb[p] = 0.0;
    });
    double kcb = 0.0;                                   // k_dot_ci . b (this lane's rows)
    static_for<0, R>([&](auto PI) { kcb = fma(u[(int)PI], bq[(int)PI], kcb); });
    static_for<0, K>([&](auto QI) {
        constexpr int q = QI, pq = q / P, rq = q % P;
        const double y0 = group_bcast<P, rq>(c0[pq]);
        const double y1 = group_bcast<P, rq>(c1[pq]);
        const double y2 = group_bcast<P, rq>(c2[pq]);
        const double bqq = group_bcast<P, rq>(bq[pq]);  // 0 for a padded neighbour
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            const double kd = kappa_dot<KIND>(sqdist3(c0[p], c1[p], c2[p], y0, y1, y2), a.cov, a.sigma_amp, a.sdot,
                                              a.ldot);
            kdb[p] = fma(kd, bqq, kdb[p]);
        });
    });
    double bkb = 0.0;
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        u[p] = ok[p] ? u[p] - kdb[p] : 0.0;
        bkb = fma(bq[p], kdb[p], bkb);
    });
    kcb = group_sum<P>(kcb);
    bkb = group_sum<P>(bkb);
    // K_cc and its Cholesky factor, then b_dot = K_cc^-1 u
    double A[NA];
    assemble_kcc<double, K, P, KIND>(c0, c1, c2, ok, r, a.cov, A);
    double Dg[R], Inv[R];
    static_for<0, R>([&](auto PI) { Dg[(int)PI] = ok[(int)PI] ? a.diag : 1.0; });
    bool bad = false;
    double minpiv = a.diag;
    cholesky_kcc<double, K, P>(A, Dg, Inv, r, bad, minpiv);
    lower_solve<double, K, P>(A, Inv, u, r);
    upper_solve<double, K, P>(A, Inv, u, r);
    const double kii_dot = a.sdot * 2.0 * a.sigma_amp;            // d kappa(0) / d sigma; d/d ell is 0
    const double sig = (double)a.sigma[sp];
    const double sdot = (kii_dot - 2.0 * kcb + bkb) / (2.0 * sig);
    if (live) {
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            a.bdot[base + (int64_t)(p * P + r) * kTile] = (TS)u[p];
        });
        if (r == 0) a.sigdot[sp] = (TS)sdot;
    }
    double ls = (live && r == 0) ? sdot / sig : 0.0;
    for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off, 64);
    __shared__ double red[kBlock / 64];
    if ((tid & 63) == 0) red[tid >> 6] = ls;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w];
        a.part[blk] = s;
    }
}

template <typename TS, int K>
hipError_t launch_tangent_factor_t(const TangentArgs<TS>& args, int kind, hipStream_t s) {
    constexpr int PTS = kBlock / factor_lanes(VECCHIA_FP64, K);
    TangentArgs<TS> a = args;
    a.nblocks = (a.ns + PTS - 1) / PTS;
    if (a.nblocks == 0) return hipSuccess;
    switch (kind) {
        case 0: hipLaunchKernelGGL((tangent_factor_kernel<TS, K, 0>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 1: hipLaunchKernelGGL((tangent_factor_kernel<TS, K, 1>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((tangent_factor_kernel<TS, K, 2>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((tangent_factor_kernel<TS, K, 3>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Untyped launch parameters of the whole tangent pass.
struct TangentLaunch {
    int precision, kp, kind, n0, n_levels;
    int64_t n, ns;
    const int32_t* level_ptr;   // host
    const void *x, *b, *sigma, *xi, *v, *xi_dot;
    const int32_t* nbr;
    const double* l0;
    void *bdot, *sigdot, *v_dot;
    double *part, *fixzero, *ld0dot, *stage, *logdet_dot;
    double diag, sigma_amp, sdot, ldot;
    vecchia_kernel kern;
};

template <int K>
hipError_t launch_tangent_factor_width(const TangentLaunch& L, hipStream_t s) {
    if (L.precision == VECCHIA_FP32) {
        TangentArgs<float> a{static_cast<const float*>(L.x), L.nbr, static_cast<const float*>(L.b),
                             static_cast<const float*>(L.sigma), static_cast<float*>(L.bdot),
                             static_cast<float*>(L.sigdot), L.part, L.ns, 0, L.n0, L.diag, L.sigma_amp, L.sdot,
                             L.ldot, make_cov<double>(L.kern)};
        return launch_tangent_factor_t<float, K>(a, L.kind, s);
    }
    TangentArgs<double> a{static_cast<const double*>(L.x), L.nbr, static_cast<const double*>(L.b),
                          static_cast<const double*>(L.sigma), static_cast<double*>(L.bdot),
                          static_cast<double*>(L.sigdot), L.part, L.ns, 0, L.n0, L.diag, L.sigma_amp, L.sdot, L.ldot,
                          make_cov<double>(L.kern)};
    return launch_tangent_factor_t<double, K>(a, L.kind, s);
}

hipError_t launch_tangent_factor_k8(const TangentLaunch& L, hipStream_t s);
hipError_t launch_tangent_factor_k16(const TangentLaunch& L, hipStream_t s);
hipError_t launch_tangent_factor_k32(const TangentLaunch& L, hipStream_t s);
hipError_t launch_tangent_factor_k64(const TangentLaunch& L, hipStream_t s);
hipError_t launch_forward_tangent(const TangentLaunch& L, hipStream_t s);

// Scratch of vecchia_forward_jvp: b_dot (tiled), sigma_dot, per-block sums
// of sigma_dot / sigma, zeros for the logdet reduction's fixed-point input,
// the dense block's trace term and the reduction's staging.
struct TangentScratch {
    size_t bdot = 0, sigdot = 0, part = 0, fixzero = 0, ld0dot = 0, stage = 0, total = 0;
    int64_t nblocks = 0;
};
inline TangentScratch tangent_scratch(int64_t n, int kp, int n0, int precision) {
    TangentScratch t;
    const int64_t ns = n - n0;
    const int64_t tiles = (ns + kTile - 1) / kTile;
    const size_t esz = precision == VECCHIA_FP64 ? 8 : 4;
    const int pts = kBlock / factor_lanes(VECCHIA_FP64, kp);
    t.nblocks = (ns + pts - 1) / pts;
    const int64_t nb = t.nblocks > 0 ? t.nblocks : 1;
    size_t off = 0;
    t.bdot = off;
    off = align256(off + (size_t)(tiles > 0 ? tiles : 1) * kp * kTile * esz);
    t.sigdot = off;
    off = align256(off + (size_t)(tiles > 0 ? tiles : 1) * kTile * esz);
    t.part = off;
    off = align256(off + (size_t)nb * sizeof(double));
    t.fixzero = off;
    off = align256(off + (size_t)nb * sizeof(double));
    t.ld0dot = off;
    off = align256(off + sizeof(double));
    t.stage = off;
    off = align256(off + 2 * 256 * sizeof(double));
    t.total = off;
    return t;
}

}  // namespace vk
