// Eq. (2) for conditioning sets of 64 neighbours: one point per wave, lane i
// owns row i of K_cc.
//
// Mapping on CDNA4.  At k = 64 the packed lower triangle holds 2080 values per
// point, more than a few lanes can keep in registers, so the point takes the
// whole wave: lane i keeps row i of L (64 doubles) in registers and the
// Cholesky is left-looking,
//     L_ij = (K_ij - sum_{m<j} L_im L_jm) / L_jj,   i > j,
// with K_ij evaluated when column j is reached (nothing of size k^2 is
// assembled first).  Row j, needed by every lane at step j, is read from a
// packed copy of L in LDS (one broadcast read of two doubles per instruction)
// that each lane fills as its entries become final.  The pivot d_j is read
// from lane j (a wave-uniform value), square-rooted and inverted in double.
// The forward substitution y = L^-1 k_ci runs down the columns with y_j taken
// from lane j; the backward substitution L^T b = y reads the rows of L from
// LDS.  Padded neighbours (-1) sit at far-away points: identity rows and
// columns of K_cc, zero entries of k_ci, as in the narrower kernels.
//
// All arithmetic is double; the storage type TS is float (FP32 path) or
// double.  Lanes i < j compute values at step j that are never used (the
// upper triangle), so three quarters of the Cholesky's lane work is useful.
#pragma once

#include "factor_kernel.h"

namespace vk {

constexpr int kWide = 64;

// Packed lower rows in LDS, each row padded to an even length so that every
// row starts on a 16-byte boundary (two doubles per read).
__host__ __device__ constexpr int wide_row_len(int i) { return (i + 2) & ~1; }
__host__ __device__ constexpr int wide_row_off(int i) {
    return i == 0 ? 0 : wide_row_off(i - 1) + wide_row_len(i - 1);
}
constexpr int kWideLdsRows = wide_row_off(kWide);        // doubles per wave
// the same offset for a row index known only at run time
__device__ __forceinline__ int wide_row_off_rt(int i) { return (i / 2) * (i / 2 + 1) * 2 + (i & 1) * ((i / 2) * 2 + 2); }
constexpr int kWideWaves = kBlock / 64;                  // points per workgroup

struct WideLds {
    double L[kWideWaves][kWideLdsRows];
    double c[kWideWaves][kWide][4];                      // neighbour coordinates (x, y, z, ok)
};

__device__ __forceinline__ double wide_readlane(double v, int lane) {
    const int64_t u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double wide_wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Gathers the coordinates of neighbour `lane` of sparse point sp into LDS and
// returns them (far-away point for padding).
template <typename TX>
__device__ __forceinline__ void wide_gather(const TX* __restrict__ x, const int32_t* __restrict__ nbr, int64_t sp,
                                            int lane, double (*c)[4], double& c0, double& c1, double& c2, bool& ok) {
    const int32_t j = nbr[(sp >> 6) * (int64_t)kWide * kTile + (int64_t)lane * kTile + (sp & 63)];
    const int64_t jj = j >= 0 ? j : 0;
    const double x0 = (double)x[jj * 3 + 0], x1 = (double)x[jj * 3 + 1], x2 = (double)x[jj * 3 + 2];
    ok = j >= 0;
    c0 = ok ? x0 : 1e15 * (double)(lane + 1);
    c1 = ok ? x1 : 0.0;
    c2 = ok ? x2 : 0.0;
    c[lane][0] = c0;
    c[lane][1] = c1;
    c[lane][2] = c2;
    c[lane][3] = ok ? 1.0 : 0.0;
}

// Left-looking Cholesky of K_cc (see above).  On return L[] holds row `lane`
// of L (strictly lower part; zero on and above the diagonal), Lds its packed
// copy, inv = 1/L_ii of this lane's row; bad / minpiv over all pivots.
template <int KIND>
__device__ __forceinline__ void wide_cholesky(double* __restrict__ Lds, const double (*c)[4], double c0, double c1,
                                              double c2, bool ok, int lane, const Cov<double>& cov, double diag,
                                              double (&L)[kWide], double& inv, bool& bad, double& minpiv) {
    const double dii = ok ? diag : 1.0;
    inv = 0.0;
    static_for<0, kWide>([&](auto JI) {
        constexpr int j = JI;
        L[j] = 0.0;
        const double y0 = c[j][0], y1 = c[j][1], y2 = c[j][2];
        double s = lane == j ? dii : cov_r2<KIND>(sqdist3(c0, c1, c2, y0, y1, y2), cov);
        constexpr int off = wide_row_off(j);
        static_for<0, j / 2>([&](auto MI) {
            constexpr int m = 2 * MI;
            const double2 lj = *reinterpret_cast<const double2*>(Lds + off + m);
            s = fma(-L[m], lj.x, s);
            s = fma(-L[m + 1], lj.y, s);
        });
        if constexpr (j % 2 == 1) s = fma(-L[j - 1], Lds[off + j - 1], s);
        const double d = wide_readlane(s, j);
        bad |= !(d > 0.0);
        minpiv = fmin(minpiv, d);
        const double invt = rsqrt_f64(d);
        inv = lane == j ? invt : inv;
        const double lij = lane > j ? s * invt : 0.0;
        L[j] = lij;
        // entry j of row `lane` is final: into the LDS copy (LDS operations of
        // one wave complete in order, so later steps read it back)
        if (lane > j) Lds[wide_row_off_rt(lane) + j] = lij;
    });
}

// y = L^-1 z (z distributed like the rows, in place), returns y.y.
__device__ __forceinline__ double wide_lower_solve(const double (&L)[kWide], double inv, int lane, double& z) {
    double yy = 0.0;
    static_for<0, kWide>([&](auto JI) {
        constexpr int j = JI;
        const double yj = wide_readlane(z, j) * wide_readlane(inv, j);
        yy = fma(yj, yj, yy);
        z = lane == j ? yj : (lane > j ? fma(-L[j], yj, z) : z);
    });
    return yy;
}

// L^T x = z in place, rows of L read from the LDS copy.
__device__ __forceinline__ void wide_upper_solve(const double* __restrict__ Lds, double inv, int lane, double& z) {
    static_for<0, kWide>([&](auto JJ) {
        constexpr int j = kWide - 1 - (int)JJ;
        const double xj = wide_readlane(z, j) * wide_readlane(inv, j);
        const double lj = Lds[wide_row_off(j) + (lane < j ? lane : 0)];
        z = lane == j ? xj : (lane < j ? fma(-lj, xj, z) : z);
    });
}

}  // namespace vk

namespace vk {

// Eq. (2) for one sparse point per wave; see the file comment.  FP32 storage
// (TS = float) keeps every point in double arithmetic: the precision policy's
// all-double branch, taken at this width without a sample.
template <typename TS, int KIND>
__global__ __launch_bounds__(kBlock) void factor_wide_kernel(FactorArgs<TS> a, Cov<double> cov) {
    __shared__ WideLds sh;
    __shared__ double part[kWideWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t blk = xcd_block(blockIdx.x, a.nblocks);
    const int64_t sp_raw = blk * kWideWaves + wave;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;
    if (sizeof(TS) == 4 && blockIdx.x == 0 && threadIdx.x == 0) a.status[2] = (uint64_t)a.ns;   // all in double
    double c0, c1, c2;
    bool ok;
    wide_gather<TS>(a.x, a.nbr, sp, lane, sh.c[wave], c0, c1, c2, ok);
    const TS* xt = a.x + (a.n0 + sp) * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];
    double L[kWide];
    double inv;
    bool bad = false;
    double minpiv = a.diag;
    wide_cholesky<KIND>(sh.L[wave], sh.c[wave], c0, c1, c2, ok, lane, cov, a.diag, L, inv, bad, minpiv);
    double z = ok ? cov_r2<KIND>(sqdist3(c0, c1, c2, t0, t1, t2), cov) : 0.0;
    const double s2 = a.diag - wide_lower_solve(L, inv, lane, z);
    wide_upper_solve(sh.L[wave], inv, lane, z);
    bad |= !(s2 > 0.0);
    if (live) {
        a.b[(sp >> 6) * (int64_t)kWide * kTile + (int64_t)lane * kTile + (sp & 63)] = (TS)z;
        if (lane == 0) {
            a.sigma[sp] = (TS)sqrt(s2);
            if (bad) {
                atomicMin((unsigned long long*)&a.status[0], (unsigned long long)(a.n0 + sp));
                atomicAdd((unsigned long long*)&a.status[1], 1ull);
            }
        }
    }
    if (lane == 0) part[wave] = (live && !bad) ? 0.5 * log(s2) : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kWideWaves; ++w) s += part[w];
        a.ldpart[blk] = s;
        a.ldfix[blk] = 0;
    }
}

template <typename TS>
hipError_t launch_factor_wide_t(const FactorLaunch& L, hipStream_t stream) {
    if (!(L.stages & kStageMain)) return hipSuccess;      // no sample and no second pass at this width
    FactorArgs<TS> a;
    a.x = static_cast<const TS*>(L.x);
    a.nbr = L.nbr;
    a.b = static_cast<TS*>(L.b);
    a.sigma = static_cast<TS*>(L.sigma);
    a.ldpart = L.ldpart;
    a.ldfix = L.ldfix;
    a.status = L.status;
    a.redo = L.redo;
    a.ns = L.ns;
    a.n0 = L.n0;
    a.cov = make_cov<TS>(L.kern);
    a.diag = L.kern.sigma * L.kern.sigma + L.kern.nugget;
    a.redo_ratio = 0.0;
    a.probe_stride = 0;
    a.nblocks = (L.ns + kWideWaves - 1) / kWideWaves;
    if (a.nblocks == 0) return hipSuccess;
    const Cov<double> cov = make_cov<double>(L.kern);
    switch (L.kind) {
        case 0: hipLaunchKernelGGL((factor_wide_kernel<TS, 0>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, stream, a, cov); break;
        case 1: hipLaunchKernelGGL((factor_wide_kernel<TS, 1>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, stream, a, cov); break;
        case 2: hipLaunchKernelGGL((factor_wide_kernel<TS, 2>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, stream, a, cov); break;
        case 3: hipLaunchKernelGGL((factor_wide_kernel<TS, 3>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, stream, a, cov); break;
        case 4: hipLaunchKernelGGL((factor_wide_kernel<TS, 4>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, stream, a, cov); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vk
