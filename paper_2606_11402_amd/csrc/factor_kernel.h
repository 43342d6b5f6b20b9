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

#include <algorithm>

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
    long long* ldfix;      // per-block sum of log sigma of the points recomputed from the list, 2^-32 fixed point
    uint64_t* status;      // [first bad position, bad count, redo count, unused, unused,
                           //  policy sample: flagged, looked at]
    uint32_t* redo;        // FP32 path: sparse indices recomputed in double
    int64_t ns;
    int64_t nblocks;
    int n0;
    Cov<T> cov;
    double diag;           // K_ii = sigma^2 + nugget, double
    double redo_ratio;     // FP32 path: recompute a point in double when a pivot < redo_ratio * K_ii
    int64_t probe_stride;  // FP32 path: > 0 for the sample pass (every probe_stride-th block)
};

// FP32 path, precision policy.  A sample pass runs the float factor on every
// kProbeStride-th block and counts, in status[5] and status[6], the points
// it would send to the double recompute and the points it looked at.  When
// more than a width-dependent fraction would go, the float pass is skipped
// and every point is computed in double, in storage order.  The fraction is
// where the float pass stops paying for itself: a double recompute driven by
// the list costs about twice the per-point time of the double pass in storage
// order (scattered points), and the float pass with its refinement costs
// nearly as much as the double pass at k <= 16 (double FMA runs at the float
// rate on CDNA4; only the exponentials and square roots are cheaper in
// float), about two thirds of it at k = 32.  The choice depends only on the
// inputs, so results stay reproducible.
constexpr int64_t kProbeStride = 256;
template <int K>
__device__ __forceinline__ bool all_points_in_double(const uint64_t* status) {
    const uint64_t flagged = status[5], sampled = status[6];
    constexpr uint64_t inv_frac = K <= 16 ? 16 : 8;   // 1/16 of the points at k <= 16, 1/8 above
    return sampled > 0 && inv_frac * flagged > sampled;
}

// Fixed-point scale of the log-sigma sums of recomputed points: integer
// additions commute, so a block's sum does not depend on the order of the
// atomics.  A block holds at most kBlock points and |log sigma| < 745 for any
// positive double variance, so a block's sum stays below 2^50 (no overflow).
constexpr double kFixScale = 4294967296.0;  // 2^32

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

// Coordinates of the neighbours of the rows this lane owns.  A padded slot
// (-1) is placed at its own far-away point (1e15 (m+1), 0, 0): its kernel
// values with every other point, real or padded, are exactly 0, so it acts
// as an identity row and column of K_cc without any masking in the
// evaluation loops (the squared distances, >= 1e30, stay finite in float).
// The loads are unconditional (a padded slot reads point 0) and the padding
// is selected afterwards: a load under a condition cannot be issued early, so
// the compiler would branch around each one and wait for it, one memory round
// trip per row instead of two for all rows.
template <typename T, typename TX, int K, int P>
__device__ __forceinline__ void gather_rows(const TX* __restrict__ x, const int32_t* __restrict__ nbr, int64_t base,
                                            int r, T* c0, T* c1, T* c2, int* ok) {
    constexpr int R = K / P;
    int32_t jv[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        jv[p] = nbr[base + (int64_t)(p * P + r) * kTile];
    });
    TX x0[R], x1[R], x2[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        const int64_t jj = jv[p] >= 0 ? jv[p] : 0;
        x0[p] = x[jj * 3 + 0];
        x1[p] = x[jj * 3 + 1];
        x2[p] = x[jj * 3 + 2];
    });
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        ok[p] = jv[p] >= 0;
        const T far = (T)(1e15 * (double)(p * P + r + 1));
        c0[p] = ok[p] ? (T)x0[p] : far;
        c1[p] = ok[p] ? (T)x1[p] : T(0);
        c2[p] = ok[p] ? (T)x2[p] : T(0);
    });
}

// K_cc into the lane's row blocks.  Entries on and above the diagonal of a
// row block receive finite kernel values too; the Cholesky zeroes them when
// their column is reached, so they never act as multipliers.
template <typename T, int K, int P, int KIND>
__device__ __forceinline__ void assemble_kcc(const T* c0, const T* c1, const T* c2, const int* ok, int r,
                                             const Cov<T>& cov, T* A) {
    constexpr int R = K / P;
    (void)ok;
    (void)r;
    static_for<0, K>([&](auto LI) {
        constexpr int l = LI, pl = l / P, rl = l % P;
        const T y0 = group_bcast<P, rl>(c0[pl]);
        const T y1 = group_bcast<P, rl>(c1[pl]);
        const T y2 = group_bcast<P, rl>(c2[pl]);
        static_for<pl, R>([&](auto PI) {
            constexpr int p = PI;
            A[row_off<P>(p) + l] = cov_r2<KIND>(sqdist3(c0[p], c1[p], c2[p], y0, y1, y2), cov);
        });
    });
}

// exp(z) for |z| <= 1 as exp(z/2)^2, exp(z/2) by its Taylor series to
// degree 14 (coefficients 1/(i! 2^i), Horner in z): within about 2 units of
// double roundoff on that interval, no range reduction.
__device__ __forceinline__ double exp_small(double z) {
    double p = 1.0 / 1428329123020800.0;                // 1/(14! 2^14)
    p = fma(p, z, 1.0 / 51011754393600.0);              // 1/(13! 2^13)
    p = fma(p, z, 1.0 / 1961990553600.0);               // 1/(12! 2^12)
    p = fma(p, z, 1.0 / 81749606400.0);
    p = fma(p, z, 1.0 / 3715891200.0);
    p = fma(p, z, 1.0 / 185794560.0);
    p = fma(p, z, 1.0 / 10321920.0);
    p = fma(p, z, 1.0 / 645120.0);
    p = fma(p, z, 1.0 / 46080.0);
    p = fma(p, z, 1.0 / 3840.0);
    p = fma(p, z, 1.0 / 384.0);
    p = fma(p, z, 1.0 / 48.0);
    p = fma(p, z, 1.0 / 8.0);
    p = fma(p, z, 0.5);
    p = fma(p, z, 1.0);
    return p * p;
}

// exp(z) for |z| <= 1/4: Taylor series to degree 12 (coefficients 1/i!,
// Horner in z).  The remainder is below e^(1/4) 4^-13 / 13! < 4e-18 relative
// and each Horner step adds at most a quarter of the previous rounding error,
// so the result is within about 2 units of double roundoff with 12 operations
// instead of the 16 of exp_small.
__device__ __forceinline__ double exp_quarter(double z) {
    double p = 1.0 / 479001600.0;                       // 1/12!
    p = fma(p, z, 1.0 / 39916800.0);                    // 1/11!
    p = fma(p, z, 1.0 / 3628800.0);
    p = fma(p, z, 1.0 / 362880.0);
    p = fma(p, z, 1.0 / 40320.0);
    p = fma(p, z, 1.0 / 5040.0);
    p = fma(p, z, 1.0 / 720.0);
    p = fma(p, z, 1.0 / 120.0);
    p = fma(p, z, 1.0 / 24.0);
    p = fma(p, z, 1.0 / 6.0);
    p = fma(p, z, 0.5);
    p = fma(p, z, 1.0);
    return fma(p, z, 1.0);
}

// K_cc of the squared-exponential kernel in product form (see factor_point).
// QUARTER: every |w|^2 of the wave is at most 1/4, so every exponent
// w_p . w_l is too (Cauchy-Schwarz) and the shorter series applies.
template <typename T, int K, int P, bool QUARTER>
__device__ __forceinline__ void assemble_kcc_se_product(const T* w0, const T* w1, const T* w2, const T* a, T* A) {
    constexpr int R = K / P;
    static_for<0, K>([&](auto LI) {
        constexpr int l = LI, pl = l / P, rl = l % P;
        const T y0 = group_bcast<P, rl>(w0[pl]);
        const T y1 = group_bcast<P, rl>(w1[pl]);
        const T y2 = group_bcast<P, rl>(w2[pl]);
        const T al = group_bcast<P, rl>(a[pl]);
        static_for<pl, R>([&](auto PI) {
            constexpr int p = PI;
            const T z = fma(w0[p], y0, fma(w1[p], y1, w2[p] * y2));
            A[row_off<P>(p) + l] = (a[p] * al) * (QUARTER ? exp_quarter(z) : exp_small(z));
        });
    });
}

// Right-looking Cholesky of K_cc in place: A receives the strictly lower
// part of L (zero elsewhere), Inv[p] = 1/L_ii of the lane's rows.  Pivots
// d_j = K_jj - sum_m L_jm^2 live in Dg (double) for both storage types.
template <typename T, int K, int P>
__device__ __forceinline__ void cholesky_kcc(T* A, double* Dg, T* Inv, int r, bool& bad, double& minpiv) {
    constexpr int R = K / P;
    static_for<0, R>([&](auto PI) { Inv[(int)PI] = T(0); });
    static_for<0, K>([&](auto JI) {
        constexpr int j = JI, pj = j / P, rj = j % P;
        const double d = group_bcast<P, rj>(Dg[pj]);
        bad |= !(d > 0.0);
        minpiv = fmin(minpiv, d);
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
}

// Eq. (2) for the sparse point sp, computed in type T from coordinates of
// type TX.  On return the lane holds b for its rows in bv[], the group holds
// sigma^2 (double), the smallest pivot and whether a pivot or the variance
// was not positive.
//
// FUSED (Alg. 1 as written, nothing stored): after y = L^-1 k_ci and sigma^2
// the point gathers its neighbours' values v[c(i)] (type TV), solves
// w = L^-1 v[c(i)] with the same factor and returns the conditional mean
// y . w = k_ic K_cc^-1 v[c(i)] = b . v[c(i)] in *mean_out; b itself is never
// formed (bv[] holds y) and there is no backward substitution.
template <typename T, typename TX, int K, int P, int KIND, bool REFINE, bool FUSED = false, typename TV = T>
__device__ __forceinline__ void factor_point(const TX* __restrict__ x, const int32_t* __restrict__ nbr, int n0,
                                             int64_t sp, int r, const Cov<T>& cov, double diag, T* bv,
                                             double& s2_out, double& minpiv_out, bool& bad_out,
                                             const TV* vfused = nullptr, double* mean_out = nullptr) {
    static_assert(!(FUSED && REFINE), "the fused forward has no refinement step");
    constexpr int R = K / P;
    constexpr int NA = P * R * (R + 1) / 2;
    const int64_t base = (sp >> 6) * (int64_t)K * kTile + (sp & 63);

    const TX* xt = x + (int64_t)(n0 + sp) * 3;
    const T t0 = (T)xt[0], t1 = (T)xt[1], t2 = (T)xt[2];
    T c0[R], c1[R], c2[R];
    int ok[R];
    gather_rows<T, TX, K, P>(x, nbr, base, r, c0, c1, c2, ok);

    T A[NA];
    T kc[R];
    double Dg[R];
    static_for<0, R>([&](auto PI) { Dg[(int)PI] = ok[(int)PI] ? diag : 1.0; });
    if constexpr (KIND == 2 && sizeof(T) == 8) {
        // Squared exponential in double, product form around the target:
        // with w = (x - t) / ell, K_pl = a_p a_l exp(w_p . w_l) and
        // a_p = sigma exp(-|w_p|^2 / 2), the target column k_p = sigma a_p.
        // A product adds no cancellation, and when every |w|^2 in the wave is
        // at most 1 the exponential of w_p . w_l is a short series (no range
        // reduction): R exponentials per lane instead of one per entry.
        // When every |w|^2 is at most 1/4 a shorter series suffices.
        // Padded neighbours get a = 0 and w = 0 (identity row and column).
        T w0[R], w1[R], w2[R], a[R];
        bool near = true, quarter = true;
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            w0[p] = ok[p] ? (c0[p] - t0) * cov.inv_ell : T(0);
            w1[p] = ok[p] ? (c1[p] - t1) * cov.inv_ell : T(0);
            w2[p] = ok[p] ? (c2[p] - t2) * cov.inv_ell : T(0);
            const T q = w0[p] * w0[p] + w1[p] * w1[p] + w2[p] * w2[p];
            near = near && q <= T(1);
            quarter = quarter && q <= T(0.25);
            a[p] = ok[p] ? cov.sigma * exp(T(-0.5) * q) : T(0);
            kc[p] = cov.sigma * a[p];
        });
        if (__all(quarter)) {
            assemble_kcc_se_product<T, K, P, true>(w0, w1, w2, a, A);
        } else if (__all(near)) {
            assemble_kcc_se_product<T, K, P, false>(w0, w1, w2, a, A);
        } else {
            assemble_kcc<T, K, P, KIND>(c0, c1, c2, ok, r, cov, A);
        }
    } else {
        assemble_kcc<T, K, P, KIND>(c0, c1, c2, ok, r, cov, A);
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            kc[p] = cov_r2<KIND>(sqdist3(c0[p], c1[p], c2[p], t0, t1, t2), cov);
        });
    }

    T Inv[R];
    bool bad = false;
    double minpiv = diag;
    cholesky_kcc<T, K, P>(A, Dg, Inv, r, bad, minpiv);

    // ---- y = L^-1 k_ci, sigma^2 = K_ii - y.y (double), b = L^-T y
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
    double s2 = diag - yy;
    if constexpr (FUSED) {
        T vc[R];
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            const int32_t j = nbr[base + (int64_t)(p * P + r) * kTile];
            const TV vj = vfused[j >= 0 ? j : 0];          // unconditional load, selected below
            vc[p] = j >= 0 ? (T)vj : T(0);
        });
        lower_solve<T, K, P>(A, Inv, vc, r);
        double dot = 0.0;
        static_for<0, R>([&](auto PI) { dot = fma((double)bv[(int)PI], (double)vc[(int)PI], dot); });
        *mean_out = group_sum<P>(dot);
        bad |= !(s2 > 0.0);
        s2_out = s2;
        minpiv_out = minpiv;
        bad_out = bad;
        return;
    }
    upper_solve<T, K, P>(A, Inv, bv, r);

    if constexpr (REFINE) {
        // Residual k_ci - K_cc b, double accumulation, K_cc recomputed.  The
        // empty asm makes the coordinates opaque after the solve, so the
        // compiler cannot reuse the kernel values of the assembly (which
        // would keep all of K_cc live in registers through the Cholesky).
#pragma unroll
        for (int p = 0; p < R; ++p) asm volatile("" : "+v"(c0[p]), "+v"(c1[p]), "+v"(c2[p]) : "v"(bv[0]));
        double res[R];
        // kappa(0) b_i enters through the l = i term of the loop; the nugget
        // part of K_ii is added here (a padded row has b_i = 0).
        const double nug = diag - (double)cov.s2;
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            res[p] = (double)kc[p] - nug * (double)bv[p];
        });
        // K_cc is symmetric: for column l the lane evaluates only its row
        // blocks p >= block(l).  Each value enters its own row (times b_l)
        // and, below the diagonal block, also row l (times the lane's b_row),
        // the latter summed over the group and added by the owner of row l.
        // Every entry of K_cc b is then counted once, with half the kernel
        // evaluations of the full product.
        static_for<0, K>([&](auto LI) {
            constexpr int l = LI, pl = l / P, rl = l % P;
            const T y0 = group_bcast<P, rl>(c0[pl]);
            const T y1 = group_bcast<P, rl>(c1[pl]);
            const T y2 = group_bcast<P, rl>(c2[pl]);
            const double bl = (double)group_bcast<P, rl>(bv[pl]);
            double col = 0.0;
            static_for<pl, R>([&](auto PI) {
                constexpr int p = PI;
                const double val = (double)cov_r2<KIND>(sqdist3(c0[p], c1[p], c2[p], y0, y1, y2), cov);
                res[p] = fma(-val, bl, res[p]);
                if constexpr (p > pl) col = fma(-val, (double)bv[p], col);
            });
            if constexpr (pl + 1 < R) {
                col = group_sum<P>(col);
                res[pl] += (r == rl) ? col : 0.0;
            }
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
        s2 = diag - group_sum<P>(kb);
    }
    bad |= !(s2 > 0.0);
    s2_out = s2;
    minpiv_out = minpiv;
    bad_out = bad;
}

// One group of P lanes per sparse point, all points at once.  FP32 storage
// (REFINE): a point whose pivots fail or fall below redo_ratio * K_ii is not
// written here; it is appended to the redo list and recomputed in double by
// factor_redo_kernel.  Each workgroup appends its points as one contiguous
// run (one atomic per workgroup), so the list keeps the storage order of
// neighbouring points and the recompute gathers stay local.  PROBE: the
// policy sample pass (counts only, writes nothing else).
template <typename T, int K, int P, int KIND, bool REFINE, bool PROBE>
__global__ __launch_bounds__(kBlock, factor_min_waves(sizeof(T), K)) void factor_sparse_kernel(FactorArgs<T> a) {
    static_assert(K % P == 0, "K must be a multiple of P");
    constexpr int R = K / P;
    constexpr int PTS = kBlock / P;
    const int tid = threadIdx.x;
    const int r = tid % P;
    constexpr bool probe = REFINE && PROBE;
    const int64_t blk = probe ? (int64_t)blockIdx.x * a.probe_stride : xcd_block(blockIdx.x, a.nblocks);
    if (REFINE && !probe && all_points_in_double<K>(a.status)) {
        if (tid == 0) {                                // every point goes to factor_redo_kernel
            a.ldpart[blk] = 0.0;
            a.ldfix[blk] = 0;
        }
        return;
    }
    const int64_t sp_raw = blk * PTS + tid / P;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;      // dead lanes mirror a live point
    const int64_t base = (sp >> 6) * (int64_t)K * kTile + (sp & 63);

    T bv[R];
    double s2, minpiv;
    bool bad;
    factor_point<T, T, K, P, KIND, REFINE>(a.x, a.nbr, a.n0, sp, r, a.cov, a.diag, bv, s2, minpiv, bad);
    const bool redo = REFINE && (bad || minpiv < a.redo_ratio * a.diag);

    if constexpr (probe) {
        __shared__ unsigned counts[2];
        if (tid == 0) counts[0] = counts[1] = 0u;
        __syncthreads();
        if (live && r == 0) {
            atomicAdd(&counts[0], redo ? 1u : 0u);
            atomicAdd(&counts[1], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            atomicAdd((unsigned long long*)&a.status[5], (unsigned long long)counts[0]);
            atomicAdd((unsigned long long*)&a.status[6], (unsigned long long)counts[1]);
        }
        return;
    }

    if (live && !redo) {
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
    if constexpr (REFINE) {
        // the workgroup's recompute points as one run: rank within the
        // workgroup by a prefix count, one atomic for the run's start
        __shared__ unsigned wave_cnt[kBlock / 64];
        __shared__ unsigned long long run_start;
        const bool mine = live && redo && r == 0;
        const uint64_t ballot = __ballot(mine);
        const int lane = tid & 63, wave = tid >> 6;
        if (lane == 0) wave_cnt[wave] = (unsigned)__popcll(ballot);
        __syncthreads();
        if (tid == 0) {
            unsigned total = 0;
            for (int w = 0; w < kBlock / 64; ++w) total += wave_cnt[w];
            run_start = total ? atomicAdd((unsigned long long*)&a.status[2], (unsigned long long)total) : 0ull;
        }
        __syncthreads();
        if (mine) {
            unsigned before = (unsigned)__popcll(ballot & ((1ull << lane) - 1ull));
            for (int w = 0; w < wave; ++w) before += wave_cnt[w];
            a.redo[run_start + before] = (uint32_t)sp;
        }
    }
    double lsum = (live && !redo && r == 0) ? 0.5 * log(s2) : 0.0;
    lsum = wave_sum_f64<T>(lsum);
    __shared__ double part[kBlock / 64];
    if ((tid & 63) == 0) part[tid >> 6] = lsum;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += part[w];
        a.ldpart[blk] = s;
        a.ldfix[blk] = 0;                              // factor_redo_kernel adds the deferred points
    }
}

// FP32 storage: the listed points again, entirely in double (kernel values,
// Cholesky, solves), results rounded to float.  The grid covers every sparse
// point (the list length is known only on the device); groups past the list
// end leave at once.  log sigma: when every point is recomputed (policy) a
// workgroup covers the same points as the float pass would and writes its
// double partial to ldpart; otherwise each point adds its term in fixed point
// to ldfix of the float-pass block it belongs to (integer atomics commute, so
// the sum is the same whatever order the list and the atomics take).
template <int K, int KIND>
__global__ __launch_bounds__(kBlock, factor_min_waves(8, K)) void factor_redo_kernel(FactorArgs<float> a,
                                                                                       Cov<double> cov) {
    constexpr int P = factor_lanes(VECCHIA_FP64, K);
    static_assert(P == factor_lanes(VECCHIA_FP32, K), "float and double passes share the block of a point");
    constexpr int R = K / P;
    constexpr int PTS = kBlock / P;
    const int tid = threadIdx.x;
    const int r = tid % P;
    const bool direct = all_points_in_double<K>(a.status);
    const int64_t count = direct ? a.ns : (int64_t)a.status[2];
    if (direct && blockIdx.x == 0 && tid == 0) a.status[2] = (uint64_t)a.ns;   // recompute count for the host
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk * PTS >= count) return;
    const int64_t e = blk * PTS + tid / P;
    double lsum = 0.0;
    if (e < count) {
        const int64_t sp = direct ? e : (int64_t)a.redo[e];
        const int64_t base = (sp >> 6) * (int64_t)K * kTile + (sp & 63);
        double bv[R];
        double s2, minpiv;
        bool bad;
        factor_point<double, float, K, P, KIND, false>(a.x, a.nbr, a.n0, sp, r, cov, a.diag, bv, s2, minpiv, bad);
        static_for<0, R>([&](auto PI) {
            constexpr int p = PI;
            a.b[base + (int64_t)(p * P + r) * kTile] = (float)bv[p];
        });
        if (r == 0) {
            a.sigma[sp] = (float)sqrt(s2);
            if (bad) {
                atomicMin((unsigned long long*)&a.status[0], (unsigned long long)(a.n0 + sp));
                atomicAdd((unsigned long long*)&a.status[1], 1ull);
            } else if (direct) {
                lsum = 0.5 * log(s2);
            } else {
                const long long f = __double2ll_rn(0.5 * log(s2) * kFixScale);
                atomicAdd((unsigned long long*)&a.ldfix[sp / PTS], (unsigned long long)f);
            }
        }
    }
    if (!direct) return;
    __shared__ double part[kBlock / 64];
    lsum = wave_sum_f64<double>(lsum);
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
    a.ldfix = L.ldfix;
    a.status = L.status;
    a.redo = L.redo;
    a.ns = L.ns;
    a.n0 = L.n0;
    a.cov = make_cov<T>(L.kern);
    a.diag = L.kern.sigma * L.kern.sigma + L.kern.nugget;
    a.redo_ratio = L.redo_ratio;
    a.probe_stride = 0;
    const int64_t pts = kBlock / P;
    a.nblocks = (L.ns + pts - 1) / pts;
    if (a.nblocks == 0) return hipSuccess;
    constexpr bool refine = sizeof(T) == 4;
    if (refine && L.redo_ratio > 0.0 && (L.stages & kStageProbe)) {
        FactorArgs<T> pa = a;
        pa.probe_stride = kProbeStride;
        const int64_t probe_blocks = (a.nblocks + kProbeStride - 1) / kProbeStride;
        hipLaunchKernelGGL((factor_sparse_kernel<T, K, P, KIND, refine, true>), dim3((unsigned)probe_blocks),
                           dim3(kBlock), 0, stream, pa);
        hipError_t pe = hipGetLastError();
        if (pe != hipSuccess) return pe;
    }
    hipError_t e = hipSuccess;
    if (L.stages & kStageMain) {
        hipLaunchKernelGGL((factor_sparse_kernel<T, K, P, KIND, refine, false>), dim3((unsigned)a.nblocks),
                           dim3(kBlock), 0, stream, a);
        e = hipGetLastError();
    }
    if (e != hipSuccess || !refine || !(L.stages & kStageRedo)) return e;
    if constexpr (refine) {
        constexpr int P64 = factor_lanes(VECCHIA_FP64, K);
        const int64_t blocks = (L.ns * P64 + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((factor_redo_kernel<K, KIND>), dim3((unsigned)blocks), dim3(kBlock), 0, stream, a,
                           make_cov<double>(L.kern));
        e = hipGetLastError();
    }
    return e;
}

}  // namespace vk
