// Sparse factor kernel: Eq. (2) for every point with a full neighbour row.
//
// For a point i with conditioning set c = c(i) (k = K neighbours, -1 padded):
//   K_cc = L L^T,  y = L^-1 k_ci,  b_i = L^-T y,  sigma_i^2 = K_ii - y.y
// (Alg. 1 writes the same quantities as the last row of the Cholesky factor
// of the joint covariance of [c(i), i]).  Padded neighbours (-1) give an
// identity row and column of K_cc and a zero entry of k_ci, which leaves b and
// sigma of the real neighbours unchanged.
//
// Mapping on CDNA4: a group of P consecutive lanes of a wave64 works on one
// point; lane r of the group owns the rows i = p*P + r (p = 0..R-1, R = K/P)
// of K_cc in registers, packed as the lower part of its rows up to the end
// of the row block (row block p holds columns 0..p*P+P-1).  A column value
// owned by another lane is read with a DPP quad permute (lanes.h), so the
// right-looking Cholesky, the two triangular solves and the kernel
// evaluation need no LDS and no global scratch.  The diagonal is kept apart
// in double (Dg): pivots d_j = K_jj - sum_m L_jm^2 are accumulated, square
// rooted and inverted in double for both precisions; 1/L_jj is kept per row
// (Inv).  Entries above the diagonal and the diagonal slot of A are zeroed
// when their column is reached, so that stale values never act as
// multipliers.
//
// FP32 path (REFINE): one step of iterative refinement of b: the residual
// k_ci - K_cc b is accumulated in double with K_cc recomputed from the
// coordinates (nothing of size k^2 is stored), the correction solves with
// the same factor, and sigma^2 = K_ii - k_ci . b is recomputed in double.
//
// Outputs: b (tiled layout), sigma, the block's sum of log sigma_i in double
// and, on a non-positive pivot or variance, the smallest failing storage
// position in status[0] (status[1] counts failing points).
#pragma once

#include "common.h"
#include "lanes.h"

namespace vk {

template <typename T>
struct FactorArgs {
    const T* x;            // N x 3, storage order
    const int32_t* nbr;    // tiled neighbour indices
    T* b;                  // tiled coefficients
    T* sigma;              // conditional standard deviation per sparse index
    double* ldpart;        // per-block sum of log sigma
    uint64_t* status;
    int64_t ns;
    int64_t nblocks;
    int n0;
    Cov<T> cov;
    double diag;           // K_ii = sigma^2 + nugget, double
};

template <int P>
__host__ __device__ constexpr int row_off(int p) {
    return P * p * (p + 1) / 2;
}

// Forward substitution L z = z (in place, z distributed like the rows).
template <typename T, int K, int P>
__device__ __forceinline__ void lower_solve(const T* A, const T* Inv, T* z, int r) {
    constexpr int R = K / P;
    static_for<0, K>([&](auto JI) {
        constexpr int j = JI, pj = j / P, rj = j % P;
        const T zj = group_bcast<P, rj>(z[pj] * Inv[pj]);
        z[pj] = (r == rj) ? zj : z[pj];
        static_for<pj, R>([&](auto PI) {
            constexpr int p = PI;
            z[p] = fma(-A[row_off<P>(p) + j], zj, z[p]);
        });
    });
}

// Backward substitution L^T z = z (in place).
template <typename T, int K, int P>
__device__ __forceinline__ void upper_solve(const T* A, const T* Inv, T* z, int r) {
    constexpr int R = K / P;
    static_for<0, K>([&](auto JJ) {
        constexpr int j = K - 1 - (int)JJ, pj = j / P, rj = j % P;
        T part = T(0);
        static_for<pj, R>([&](auto PI) {
            constexpr int p = PI;
            part = fma(A[row_off<P>(p) + j], z[p], part);
        });
        const T tot = group_sum<P>(part);
        const T zj = (z[pj] - tot) * Inv[pj];
        z[pj] = (r == rj) ? zj : z[pj];
    });
}

template <typename T>
__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T, int K, int P, int KIND, bool REFINE>
__global__ __launch_bounds__(kBlock) void factor_sparse_kernel(FactorArgs<T> a) {
    static_assert(K % P == 0, "K must be a multiple of P");
    constexpr int R = K / P;
    constexpr int NA = P * R * (R + 1) / 2;
    constexpr int PTS = kBlock / P;

    const int tid = threadIdx.x;
    const int r = tid % P;
    const int64_t blk = xcd_block(blockIdx.x, a.nblocks);
    const int64_t sp_raw = blk * PTS + tid / P;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;      // dead lanes mirror a live point
    const int64_t base = (sp >> 6) * (int64_t)K * kTile + (sp & 63);

    // ---- gather: the point, and the neighbours of the rows this lane owns
    const T* xt = a.x + (int64_t)(a.n0 + sp) * 3;
    const T t0 = xt[0], t1 = xt[1], t2 = xt[2];
    T c0[R], c1[R], c2[R];
    int ok[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        const int32_t j = a.nbr[base + (int64_t)(p * P + r) * kTile];
        ok[p] = j >= 0;
        const int64_t jj = j >= 0 ? j : 0;
        c0[p] = a.x[jj * 3 + 0];
        c1[p] = a.x[jj * 3 + 1];
        c2[p] = a.x[jj * 3 + 2];
    });

    // ---- assemble the strictly lower part of K_cc, k_ci and the diagonal
    T A[NA];
    static_for<0, K>([&](auto LI) {
        constexpr int l = LI, pl = l / P, rl = l % P;
        const T y0 = group_bcast<P, rl>(c0[pl]);
        const T y1 = group_bcast<P, rl>(c1[pl]);
        const T y2 = group_bcast<P, rl>(c2[pl]);
        const int okl = group_bcast<P, rl>(ok[pl]);
        static_for<pl, R>([&](auto PI) {
            constexpr int p = PI;
            const T val = cov_r2<KIND>(sqdist3(c0[p], c1[p], c2[p], y0, y1, y2), a.cov);
            const bool keep = (ok[p] & okl & (int)(l < p * P + r)) != 0;
            A[row_off<P>(p) + l] = keep ? val : T(0);
        });
    });
    T kc[R];
    double Dg[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        const T val = cov_r2<KIND>(sqdist3(c0[p], c1[p], c2[p], t0, t1, t2), a.cov);
        kc[p] = ok[p] ? val : T(0);
        Dg[p] = ok[p] ? a.diag : 1.0;
    });

    // ---- right-looking Cholesky of K_cc with double pivots
    T Inv[R];
    bool bad = false;
    static_for<0, R>([&](auto PI) { Inv[(int)PI] = T(0); });
    static_for<0, K>([&](auto JI) {
        constexpr int j = JI, pj = j / P, rj = j % P;
        const double d = group_bcast<P, rj>(Dg[pj]);
        bad |= !(d > 0.0);
        const T invt = (T)rsqrt_f64(d);
        Inv[pj] = (r == rj) ? invt : Inv[pj];
        static_for<pj, R>([&](auto PI) {
            constexpr int p = PI;
            T e = A[row_off<P>(p) + j];
            if constexpr (p == pj) {
                e = (r > rj) ? e * invt : T(0);
            } else {
                e = e * invt;
            }
            A[row_off<P>(p) + j] = e;
            const double ed = (double)e;
            Dg[p] = fma(-ed, ed, Dg[p]);
        });
        static_for<j + 1, K>([&](auto LI) {
            constexpr int l = LI, pl = l / P, rl = l % P;
            const T cl = group_bcast<P, rl>(A[row_off<P>(pl) + j]);
            static_for<pl, R>([&](auto PI) {
                constexpr int p = PI;
                A[row_off<P>(p) + l] = fma(-A[row_off<P>(p) + j], cl, A[row_off<P>(p) + l]);
            });
        });
    });

    // ---- y = L^-1 k_ci, sigma^2 = K_ii - y.y (double), b = L^-T y
    T bv[R];
    static_for<0, R>([&](auto PI) { bv[(int)PI] = kc[(int)PI]; });
    double yy = 0.0;
    static_for<0, K>([&](auto JI) {
        constexpr int j = JI, pj = j / P, rj = j % P;
        const T yj = group_bcast<P, rj>(bv[pj] * Inv[pj]);
        yy = fma((double)yj, (double)yj, yy);
        bv[pj] = (r == rj) ? yj : bv[pj];
        static_for<pj, R>([&](auto PI) {
            constexpr int p = PI;
            bv[p] = fma(-A[row_off<P>(p) + j], yj, bv[p]);
        });
    });
    double s2 = a.diag - yy;
    upper_solve<T, K, P>(A, Inv, bv, r);

    if constexpr (REFINE) {
        // Residual k_ci - K_cc b, double accumulation, K_cc recomputed.  The
        // empty asm makes the coordinates opaque after the solve, so the
        // compiler cannot reuse the kernel values of the assembly (which
        // would keep all of K_cc live in registers through the Cholesky).
#pragma unroll
        for (int p = 0; p < R; ++p) asm volatile("" : "+v"(c0[p]), "+v"(c1[p]), "+v"(c2[p]) : "v"(bv[0]));
        double res[R];
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            res[p] = (double)kc[p] - (ok[p] ? a.diag : 1.0) * (double)bv[p];
        });
        static_for<0, K>([&](auto LI) {
            constexpr int l = LI, pl = l / P, rl = l % P;
            const T y0 = group_bcast<P, rl>(c0[pl]);
            const T y1 = group_bcast<P, rl>(c1[pl]);
            const T y2 = group_bcast<P, rl>(c2[pl]);
            const int okl = group_bcast<P, rl>(ok[pl]);
            const double bl = (double)group_bcast<P, rl>(bv[pl]);
            static_for<0, R>([&](auto PI) {
                constexpr int p = PI;
                const T val = cov_r2<KIND>(sqdist3(c0[p], c1[p], c2[p], y0, y1, y2), a.cov);
                const bool keep = (ok[p] & okl & (int)(l != p * P + r)) != 0;
                res[p] = fma(-(double)(keep ? val : T(0)), bl, res[p]);
            });
        });
        T dz[R];
        static_for<0, R>([&](auto PI) { dz[(int)PI] = (T)res[(int)PI]; });
        lower_solve<T, K, P>(A, Inv, dz, r);
        upper_solve<T, K, P>(A, Inv, dz, r);
        double kb = 0.0;
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            bv[p] = bv[p] + dz[p];
            kb = fma((double)kc[p], (double)bv[p], kb);
        });
        s2 = a.diag - group_sum<P>(kb);
    }
    bad |= !(s2 > 0.0);

    // ---- outputs
    if (live) {
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            a.b[base + (int64_t)(p * P + r) * kTile] = bv[p];
        });
        if (r == 0) {
            a.sigma[sp] = (T)sqrt(s2);
            if (bad) {
                atomicMin((unsigned long long*)&a.status[0], (unsigned long long)(a.n0 + sp));
                atomicAdd((unsigned long long*)&a.status[1], 1ull);
            }
        }
    }
    double lsum = (live && r == 0) ? 0.5 * log(s2) : 0.0;
    lsum = wave_sum_f64<T>(lsum);
    __shared__ double part[kBlock / 64];
    if ((tid & 63) == 0) part[tid >> 6] = lsum;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += part[w];
        a.ldpart[blk] = s;
    }
}

template <typename T, int K, int KIND>
hipError_t launch_factor_sparse_t(const FactorLaunch& L, hipStream_t stream) {
    constexpr int P = factor_lanes(sizeof(T) == 4 ? VECCHIA_FP32 : VECCHIA_FP64, K);
    static_assert(kBlock % P == 0, "block");
    FactorArgs<T> a;
    a.x = static_cast<const T*>(L.x);
    a.nbr = L.nbr;
    a.b = static_cast<T*>(L.b);
    a.sigma = static_cast<T*>(L.sigma);
    a.ldpart = L.ldpart;
    a.status = L.status;
    a.ns = L.ns;
    a.n0 = L.n0;
    a.cov = make_cov<T>(L.kern);
    a.diag = L.kern.sigma * L.kern.sigma + L.kern.nugget;
    const int64_t pts = kBlock / P;
    a.nblocks = (L.ns + pts - 1) / pts;
    if (a.nblocks == 0) return hipSuccess;
    constexpr bool refine = sizeof(T) == 4;
    hipLaunchKernelGGL((factor_sparse_kernel<T, K, P, KIND, refine>), dim3((unsigned)a.nblocks), dim3(kBlock), 0,
                       stream, a);
    return hipGetLastError();
}

}  // namespace vk
