// Shared definitions of the HIP side: covariance evaluation, workspace layout
// and launch plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "vecchia.h"

namespace vk {

constexpr int kBlock = 256;           // threads per workgroup of the point kernels
constexpr int kTile = 64;             // points per tile of the tiled layout
constexpr uint64_t kStatusNone = ~0ull;

// Lanes per point of the factor kernels, by precision and padded width.
// Lane r of a group owns rows r, r+P, ...; the packed lower triangle of K_cc
// (P*R*(R+1)/2 values per lane, R = kp/P) stays in registers.  Groups of 4
// exchange values with DPP quad permutes (VALU); FP64 at kp = 32 also uses 4
// lanes, which needs the accumulation registers of one wave per SIMD (groups
// of 8 would need ds_swizzle round trips through the LDS unit instead).  At
// kp = 64 four lanes would hold 528 values each, so a point takes a whole
// wave (lane i owns row i, factor_wide.h).  Both precisions use the same P at
// every width, so the float and the double passes put a point in the same
// block.
__host__ __device__ constexpr int factor_lanes(int precision, int kp) {
    return kp <= 8 ? 1 : (kp <= 32 ? 4 : 64);
}

// Waves per SIMD that the register allocation of a factor kernel must allow.
__host__ __device__ constexpr int factor_min_waves(int elem_bytes, int kp) {
    return elem_bytes == 8 && kp == 32 ? 1 : 2;
}

// Device workspace holding one factor.  Offsets are 256-byte aligned.
struct Layout {
    int64_t ns = 0, ntiles = 0, nparts = 0;
    size_t esz = 0;
    size_t b = 0, sigma = 0, l0 = 0, ldpart = 0, ldfix = 0, ld0 = 0, ldstage = 0, status = 0, redo = 0, total = 0;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout workspace_layout(int64_t n, int kp, int n0, int precision) {
    Layout w;
    w.ns = n - n0;
    w.ntiles = (w.ns + kTile - 1) / kTile;
    w.esz = precision == VECCHIA_FP64 ? 8 : 4;
    const int pts_per_block = kBlock / factor_lanes(precision, kp);
    w.nparts = (w.ns + pts_per_block - 1) / pts_per_block;
    size_t off = 0;
    w.b = off;
    off = align256(off + (size_t)w.ntiles * kp * kTile * w.esz);
    w.sigma = off;
    off = align256(off + (size_t)w.ntiles * kTile * w.esz);
    w.l0 = off;
    off = align256(off + (size_t)n0 * n0 * sizeof(double));
    w.ldpart = off;
    off = align256(off + (size_t)(w.nparts > 0 ? w.nparts : 1) * sizeof(double));
    w.ldfix = off;
    off = align256(off + (size_t)(w.nparts > 0 ? w.nparts : 1) * sizeof(int64_t));
    w.ld0 = off;
    off = align256(off + sizeof(double));
    w.ldstage = off;
    off = align256(off + 2 * 256 * sizeof(double));
    w.status = off;
    off = align256(off + 8 * sizeof(uint64_t));
    w.redo = off;
    if (precision == VECCHIA_FP32) off = align256(off + (size_t)(w.ns > 0 ? w.ns : 1) * sizeof(uint32_t));
    w.total = off;
    return w;
}

// Device workspace of the fused forward (Alg. 1 with nothing stored per
// point): L0, the per-tile log-sigma sums (ldpart zero, ldfix fixed point,
// adjacent so that one fill clears both), the logdet staging and the status.
struct FusedLayout {
    int64_t ns = 0, ntiles = 0;
    size_t l0 = 0, ld0 = 0, ldpart = 0, ldfix = 0, ldstage = 0, status = 0, total = 0;
};

inline FusedLayout fused_layout(int64_t n, int n0) {
    FusedLayout w;
    w.ns = n - n0;
    w.ntiles = w.ns > 0 ? (w.ns + kTile - 1) / kTile : 1;
    size_t off = 0;
    w.l0 = off;
    off = align256(off + (size_t)n0 * n0 * sizeof(double));
    w.ld0 = off;
    off = align256(off + sizeof(double));
    w.ldpart = off;
    off += (size_t)w.ntiles * sizeof(double);
    w.ldfix = off;
    off = align256(off + (size_t)w.ntiles * sizeof(int64_t));
    w.ldstage = off;
    off = align256(off + 2 * 256 * sizeof(double));
    w.status = off;
    off = align256(off + 8 * sizeof(uint64_t));
    w.total = off;
    return w;
}

// Constants of the general Matern kernel (kind 4) for one nu, formed on the
// host: nu = n + mu with n = floor(nu + 1/2), mu in [-1/2, 1/2); K_mu and
// K_(mu+1) come from Temme's series or the continued fraction (see
// matern_corr), which need 1/Gamma(1 +- mu), their half difference over mu
// (gam1) and half sum (gam2), and mu pi / sin(mu pi).
struct MaternNu {
    double nu, mu;
    int n;
    double gpl, gmi;   // 1/Gamma(1 + mu), 1/Gamma(1 - mu)
    double gam1, gam2;
    double fact;       // mu pi / sin(mu pi)
    double pref;       // 2^(1 - nu) / Gamma(nu)
    double c;          // sqrt(2 nu) / ell
};

inline MaternNu make_matern(double nu, double ell) {
    MaternNu m{};
    if (!(nu > 0.0)) return m;
    m.nu = nu;
    m.n = (int)std::floor(nu + 0.5);
    m.mu = nu - m.n;
    const long double mu = m.mu;
    m.gpl = (double)(1.0L / std::tgammal(1.0L + mu));
    m.gmi = (double)(1.0L / std::tgammal(1.0L - mu));
    m.gam2 = 0.5 * (m.gpl + m.gmi);
    if (std::fabs(m.mu) < 1e-4) {
        // 1/Gamma(1 + z) = 1 + g1 z + g2 z^2 + g3 z^3 + ..., from
        // log Gamma(1 + z) = -gamma z + sum_k>=2 (-1)^k zeta(k) z^k / k:
        // g1 = gamma, g3 = zeta(3)/3 - gamma zeta(2)/2 + gamma^3/6, and
        // gam1 = -(g1 + g3 mu^2 + O(mu^4))
        const double g = 0.5772156649015329, z2 = 1.6449340668482264, z3 = 1.2020569031595943;
        const double g3 = z3 / 3.0 - g * z2 / 2.0 + g * g * g / 6.0;
        m.gam1 = -(g + g3 * m.mu * m.mu);
    } else {
        m.gam1 = (double)((1.0L / std::tgammal(1.0L - mu) - 1.0L / std::tgammal(1.0L + mu)) / (2.0L * mu));
    }
    const double pi = 3.141592653589793;
    m.fact = std::fabs(m.mu) < 1e-12 ? 1.0 : m.mu * pi / std::sin(m.mu * pi);
    m.pref = std::exp((1.0 - nu) * 0.6931471805599453 - std::lgamma(nu));
    m.c = std::sqrt(2.0 * nu) / ell;
    return m;
}

// Covariance parameters, pre-scaled on the host.  The e_* constants carry a
// factor log2(e) so that float kernel values use the hardware exp2; sigma^2
// enters the float exponential as its base-2 logarithm (one rounding of the
// argument instead of a multiply after the exp2).
template <typename T>
struct Cov {
    T s2;          // sigma^2
    T sigma;       // sigma
    T ls2;         // log2(sigma^2)
    T m32_lin;     // -ln(2) sigma^2: sigma^2 (1 + a) = sigma^2 + m32_lin * (-a log2(e))
    T inv_ell;     // 1/ell
    T c_m32;       // sqrt(3)/ell
    T c_m52;       // sqrt(5)/ell
    T c_se;        // -1/(2 ell^2)
    T e_exp;       // -log2(e)/ell
    T e_m32;       // -sqrt(3) log2(e)/ell
    T e_m52;       // -sqrt(5) log2(e)/ell
    T e_se;        // -log2(e)/(2 ell^2)
    MaternNu mat;  // kind 4 only
};

template <typename T>
inline Cov<T> make_cov(const vecchia_kernel& k) {
    const double log2e = 1.4426950408889634, sqrt3 = 1.7320508075688772;
    Cov<T> c;
    c.s2 = (T)(k.sigma * k.sigma);
    c.sigma = (T)k.sigma;
    c.ls2 = (T)std::log2(k.sigma * k.sigma);
    c.m32_lin = (T)(-0.6931471805599453 * k.sigma * k.sigma);
    c.inv_ell = (T)(1.0 / k.ell);
    c.c_m32 = (T)(sqrt3 / k.ell);
    c.c_m52 = (T)(2.23606797749979 / k.ell);
    c.c_se = (T)(-0.5 / (k.ell * k.ell));
    c.e_exp = (T)(-log2e / k.ell);
    c.e_m32 = (T)(-sqrt3 * log2e / k.ell);
    c.e_m52 = (T)(-2.23606797749979 * log2e / k.ell);
    c.e_se = (T)(-0.5 * log2e / (k.ell * k.ell));
    c.mat = make_matern(k.kind == 4 ? k.nu : 0.0, k.ell);
    return c;
}

// The Matern correlation 2^(1 - nu)/Gamma(nu) x^nu K_nu(x) (1 at x = 0).
// K_mu and K_(mu+1) for x <= 2 by Temme's series (N. M. Temme, J. Comput.
// Phys. 19, 1975): K_mu = sum_k c_k f_k and K_(mu+1) = (2/x) sum_k c_k
// (p_k - k f_k), c_k = (x^2/4)^k / k!, with f_k = (k f_(k-1) + p_(k-1) +
// q_(k-1)) / (k^2 - mu^2), p_k = p_(k-1)/(k - mu), q_k = q_(k-1)/(k + mu) from
// p_0 = (x/2)^-mu Gamma(1 + mu)/2, q_0 = (x/2)^mu Gamma(1 - mu)/2 and
// f_0 = fact (gam1 cosh(s) + gam2 ln(2/x) sinh(s)/s), s = mu ln(2/x); for
// x > 2 by Steed's evaluation of the continued fraction of Thompson and
// Barnett (J. Comput. Phys. 64, 1986) for K_(mu+1)/K_mu together with the
// series that normalises K_mu.  Then K_(m+1) = K_(m-1) + (2m/x) K_m upward
// to nu.  Relative error about 1e-13 for nu in [1/4, 8] (the sums stop at
// a relative increment of 1e-16).
static __device__ __noinline__ double matern_corr(double x, double nu, double mu, int n, double gpl, double gmi,
                                           double gam1, double gam2, double fact, double pref) {
    if (!(x > 0.0)) return 1.0;
    constexpr double eps = 1e-16;
    double k0, k1;                                  // K_mu(x), K_(mu+1)(x)
    if (x <= 2.0) {
        const double lg = log(2.0 / x);
        const double s = mu * lg;
        const double shs = fabs(s) < 1e-10 ? 1.0 : sinh(s) / s;
        double f = fact * (gam1 * cosh(s) + gam2 * lg * shs);
        const double es = exp(s);
        double p = 0.5 * es / gpl, q = 0.5 / (es * gmi);
        double ck = 1.0, sum = f, sum1 = p;
        const double x24 = 0.25 * x * x;
        for (int k = 1; k < 400; ++k) {
            const double dk = (double)k;
            f = (dk * f + p + q) / (dk * dk - mu * mu);
            ck *= x24 / dk;
            p /= dk - mu;
            q /= dk + mu;
            const double t = ck * f;
            sum += t;
            sum1 += ck * (p - dk * f);
            if (fabs(t) < eps * fabs(sum)) break;
        }
        k0 = sum;
        k1 = sum1 * 2.0 / x;
    } else {
        const double a1 = 0.25 - mu * mu;
        double b = 2.0 * (1.0 + x), d = 1.0 / b, h = d, dh = d;
        double q1 = 0.0, q2 = 1.0, qs = a1, ck = a1, an = -a1;
        double s = 1.0 + qs * dh;
        for (int i = 2; i < 1000; ++i) {
            an -= 2.0 * (i - 1);
            ck = -an * ck / i;
            const double qn = (q1 - b * q2) / an;
            q1 = q2;
            q2 = qn;
            qs += ck * qn;
            b += 2.0;
            d = 1.0 / (b + an * d);
            dh = (b * d - 1.0) * dh;
            h += dh;
            const double ds = qs * dh;
            s += ds;
            if (fabs(ds) < eps * fabs(s)) break;
        }
        k0 = sqrt(3.141592653589793 / (2.0 * x)) * exp(-x) / s;
        k1 = k0 * (mu + x + 0.5 - a1 * h) / x;
    }
    double kn = k0;
    if (n > 0) {
        kn = k1;
        for (int j = 1; j < n; ++j) {
            const double kk = k0 + 2.0 * (mu + j) / x * k1;
            k0 = k1;
            k1 = kk;
        }
        kn = k1;
    }
    return pref * exp(nu * log(x)) * kn;
}

// 1/sqrt(d) in double: hardware estimate plus one Newton-Raphson step,
// y1 = y0 + y0 (1 - d y0^2) / 2, which squares the relative error of y0.
__device__ __forceinline__ double rsqrt_f64(double d) {
    const double y0 = __builtin_amdgcn_rsq(d);
    const double e = fma(-d, y0 * y0, 1.0);
    return fma(0.5 * y0, e, y0);
}

// kappa(r) from the squared distance r2 (no nugget).  Float: hardware exp2
// and square root (about 1 ulp each); double: the device math library.
template <int KIND>
__device__ __forceinline__ float cov_r2(float r2, const Cov<float>& c) {
    static_assert(KIND >= 0 && KIND <= 3, "the general Matern kernel (kind 4) is evaluated in double only");
    if constexpr (KIND == 0) {
        return __builtin_amdgcn_exp2f(__builtin_fmaf(__builtin_amdgcn_sqrtf(r2), c.e_exp, c.ls2));
    } else if constexpr (KIND == 1) {
        const float t = __builtin_amdgcn_sqrtf(r2) * c.e_m32;            // -a log2(e)
        return __builtin_fmaf(t, c.m32_lin, c.s2) * __builtin_amdgcn_exp2f(t);
    } else if constexpr (KIND == 3) {
        const float r = __builtin_amdgcn_sqrtf(r2);
        const float a = r * c.c_m52;                                      // sqrt(5) r / ell
        const float poly = __builtin_fmaf(a, __builtin_fmaf(a, 1.0f / 3.0f, 1.0f), 1.0f);
        return c.s2 * poly * __builtin_amdgcn_exp2f(r * c.e_m52);
    } else {
        return __builtin_amdgcn_exp2f(__builtin_fmaf(r2, c.e_se, c.ls2));
    }
}

template <int KIND>
__device__ __forceinline__ double cov_r2(double r2, const Cov<double>& c) {
    if constexpr (KIND == 0) {
        return c.s2 * exp(-sqrt(r2) * c.inv_ell);
    } else if constexpr (KIND == 1) {
        const double a = sqrt(r2) * c.c_m32;
        return c.s2 * (1.0 + a) * exp(-a);
    } else if constexpr (KIND == 3) {
        const double a = sqrt(r2) * c.c_m52;
        return c.s2 * fma(a, fma(a, 1.0 / 3.0, 1.0), 1.0) * exp(-a);
    } else if constexpr (KIND == 4) {
        const MaternNu& m = c.mat;
        return c.s2 * matern_corr(sqrt(r2) * m.c, m.nu, m.mu, m.n, m.gpl, m.gmi, m.gam1, m.gam2, m.fact, m.pref);
    } else {
        return c.s2 * exp(r2 * c.c_se);
    }
}

template <typename T>
__device__ __forceinline__ T sqdist3(T a0, T a1, T a2, T b0, T b1, T b2) {
    const T d0 = a0 - b0, d1 = a1 - b1, d2 = a2 - b2;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

}  // namespace vk

// Launchers implemented in the .hip files (all enqueue on `stream`).
namespace vk {
struct FactorLaunch {
    int precision, kp, kind;
    int64_t n, ns;
    int n0;
    const void* x;
    const int32_t* nbr;
    void* b;
    void* sigma;
    double* ldpart;
    long long* ldfix;
    uint64_t* status;
    uint32_t* redo;
    double redo_ratio;
    vecchia_kernel kern;
    int stages;            // bit mask of kStage* launched by this call
};
constexpr int kStageProbe = 1, kStageMain = 2, kStageRedo = 4;   // FP32: sample, float pass, double pass
hipError_t launch_factor_sparse(const FactorLaunch& a, hipStream_t stream);
hipError_t launch_factor_dense(int precision, int kind, const void* x, int n0, const vecchia_kernel& kern,
                               double* l0, double* ld0, uint64_t* status, hipStream_t stream);
struct BackwardLaunch {
    int precision, kp, n0, n_levels;
    int64_t n, ns;
    const int32_t* level_ptr;   // host
    const void *x, *xi, *v, *vbar, *xibar_in, *b, *sigma;
    const int32_t* nbr;
    const int64_t* child_ptr;
    const int32_t* child;
    const double* l0;
    void *w, *xibar, *vbar_out;
    double *t0, *theta_part, *theta_dense, *theta_out;
    double ldbar;
    vecchia_kernel kern;
};
hipError_t launch_backward(const BackwardLaunch& p, hipStream_t stream);
// The coordinates' cotangent (N x 3 double, storage order) for the same
// cotangents; contrib: scratch of ceil(Ns/64) x kp x 64 records of 3 doubles
// (one per neighbour entry, in the entries' tiled order).
hipError_t launch_backward_x(const BackwardLaunch& p, double* xgrad, double* contrib, hipStream_t stream);

// Scratch of vecchia_backward: w (N doubles), t0 (n0 doubles), theta partials
// (2 doubles per block of the theta kernel), dense theta (2 doubles).
struct BackwardScratch {
    size_t w = 0, t0 = 0, part = 0, dense = 0, total = 0;
    int64_t nblocks = 0;
};
// Scratch of vecchia_backward_x: that of vecchia_backward, the sweep's and
// the inverse's per-point outputs (N each, storage type) and the per-entry
// coordinate contributions (ceil(Ns/64) x kp x 64 records of 3 doubles).
struct BackwardXScratch {
    size_t xibar = 0, vbar = 0, contrib = 0, total = 0;
};
inline BackwardScratch backward_scratch(int64_t n, int kp, int n0, int precision) {
    (void)precision;   // the sweep keeps w in double for both storage precisions
    BackwardScratch b;
    const int64_t ns = n - n0;
    const int pts = kBlock / factor_lanes(VECCHIA_FP64, kp);
    b.nblocks = (ns + pts - 1) / pts;
    size_t off = 0;
    b.w = off;
    off = align256(off + (size_t)n * sizeof(double));
    b.t0 = off;
    off = align256(off + (size_t)n0 * sizeof(double));
    b.part = off;
    off = align256(off + (size_t)(b.nblocks > 0 ? b.nblocks : 1) * 2 * sizeof(double));
    b.dense = off;
    off = align256(off + 2 * sizeof(double));
    b.total = off;
    return b;
}

inline BackwardXScratch backward_x_scratch(int64_t n, int kp, int n0, int precision) {
    BackwardXScratch x;
    const size_t esz = precision == VECCHIA_FP32 ? 4 : 8;
    const int64_t ntiles = (n - n0 + kTile - 1) / kTile;
    size_t off = backward_scratch(n, kp, n0, precision).total;
    x.xibar = off;
    off = align256(off + (size_t)n * esz);
    x.vbar = off;
    off = align256(off + (size_t)n * esz);
    x.contrib = off;
    off = align256(off + 3 * (size_t)(ntiles > 0 ? ntiles : 1) * kp * kTile * sizeof(double));
    x.total = off;
    return x;
}

constexpr int kLogdetStage = 256;   // first-stage workgroups of the logdet reduction
// Sets n 64-bit words to zero with a kernel (no memset node if the stream is captured).
hipError_t launch_zero_u64(void* p, int64_t n, hipStream_t stream);
// log det = 2 (sum_i (ldpart[i] + 2^-32 ldfix[i]) + ld0), compensated, fixed order.
hipError_t launch_logdet(const double* ldpart, const long long* ldfix, int64_t nparts, const double* ld0,
                         double* stage, double* out, hipStream_t stream);
}  // namespace vk
