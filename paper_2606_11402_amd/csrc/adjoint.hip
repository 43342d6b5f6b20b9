// Reverse-mode derivatives of forward, inverse and logdet (Sec. 2.3: forward
// and backward derivatives with respect to the kernel parameters).
//
// With F = (I - B)^-1 D (B strictly lower, row i = b_i at the columns c(i);
// D = diag(sigma); the dense block folded in as (I - B0)^-1 D0 = L0):
//   forward  v = F xi, cotangent vbar:  w = (I - B)^-T vbar by a reverse
//            sweep over the batches (children lists, a gather: deterministic),
//            xibar_i = sigma_i w_i, xibar0 = L0^T w0;
//   inverse  xi = F^-1 v, cotangent xibar: z = xibar / sigma,
//            vbar = (I - B)^T z, plus L0^-T xibar0 on the dense block;
//   logdet   cotangent ldbar: sigma_bar_i += 2 ldbar / sigma_i, K0bar += ldbar K0^-1.
// Per sparse point, with omega_i = w_i - z_i, bbar_i = omega_i v[c(i)],
// sigma_bar_i = omega_i xi_i + 2 ldbar/sigma_i, sbar = sigma_bar_i/(2 sigma_i)
// and u = K_cc^-1 bbar (K_cc and its Cholesky factor recomputed, nothing of
// size k^2 stored):
//   theta_bar += sbar dK_ii + sum_p (u_p - 2 sbar b_p) dk_p
//                + sum_{p,q} (sbar b_p - u_p) b_q dK_pq        (theta = sigma, ell)
// The dense block uses the Cholesky adjoint: with gamma = w0 - L0^-T xibar0,
// h = L0^T gamma, M = Phi(h xi0^T) + ldbar I (lower triangle, diagonal
// halved), theta_bar += sum_pq (L0^-T M L0^-1)_pq dK0_pq.
// All theta sums are accumulated in double and reduced in a fixed order.
#include "adjoint.h"

namespace vk {

// ---- reverse sweep of one batch: w_j = vbar_j + sum_children b w_child.
// A group of G lanes serves one node: lane t takes the children t, t + G, ...
// and the group sums its parts in a fixed butterfly, so the result does not
// depend on timing.  Child counts fall from a few hundred in the first, small
// batches to a few in the last, large ones; the host picks G per batch from
// its size so that the longest list of a batch takes a few rounds of
// gathers instead of hundreds.
template <typename TS, int KP, int G>
__global__ __launch_bounds__(kBlock) void adj_sweep_kernel(AdjArgs<TS> a, int64_t j_begin, int64_t j_end) {
    static_assert(kBlock % G == 0, "a group never straddles workgroups");
    constexpr int SH = KP == 8 ? 3 : (KP == 16 ? 4 : (KP == 32 ? 5 : 6));
    const int64_t j = j_begin + ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
    const int t = threadIdx.x % G;
    const bool live = j < j_end;                   // the same for the whole group
    const int64_t jj = live ? j : j_end - 1;       // dead groups mirror a live node and write nothing
    const int64_t e1 = a.child_ptr[jj + 1];
    double acc = 0.0;
    // four children per round: their indices, then their b and w, are loaded
    // together (past the end the loads repeat a valid child and add nothing),
    // and added in list order
    for (int64_t e = a.child_ptr[jj] + t; e < e1; e += 4 * G) {
        int32_t pk[4];
        static_for<0, 4>([&](auto U) {
            const int64_t eu = e + (int)U * G;
            pk[(int)U] = a.child[eu < e1 ? eu : e];
        });
        static_for<0, 4>([&](auto U) {
            const int64_t sp = pk[(int)U] >> SH;
            const int m = pk[(int)U] & (KP - 1);
            const double t_bw = fma((double)a.b[((sp >> 6) * KP + m) * kTile + (sp & 63)], a.w[a.n0 + sp], acc);
            acc = e + (int)U * G < e1 ? t_bw : acc;
        });
    }
    acc = group_sum<G>(acc) + (double)a.vbar[jj];
    if (live && t == 0) {
        a.w[j] = acc;
        if (j >= a.n0) a.xibar[j] = (TS)((double)a.sigma[j - a.n0] * acc);
    }
}

template <typename TS, int KP>
static hipError_t launch_adj_sweep(const AdjArgs<TS>& a, int64_t j0, int64_t j1, hipStream_t s) {
    const int64_t nodes = j1 - j0;
    auto go = [&](auto GI) {
        constexpr int G = decltype(GI)::value;
        hipLaunchKernelGGL((adj_sweep_kernel<TS, KP, G>), dim3((unsigned)((nodes * G + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, a, j0, j1);
        return hipGetLastError();
    };
    if (nodes <= 4096) return go(std::integral_constant<int, 64>{});
    if (nodes <= 65536) return go(std::integral_constant<int, 16>{});
    return go(std::integral_constant<int, 4>{});
}

// ---- inverse part: vbar_j = z_j - sum_children b z_child, z = xibar / sigma
template <typename TS, int KP>
__global__ __launch_bounds__(kBlock) void adj_inverse_kernel(AdjArgs<TS> a) {
    constexpr int SH = KP == 8 ? 3 : (KP == 16 ? 4 : (KP == 32 ? 5 : 6));
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= a.n) return;
    double acc = j >= a.n0 ? (double)a.xibar_in[j] / (double)a.sigma[j - a.n0] : 0.0;
    for (int64_t e = a.child_ptr[j]; e < a.child_ptr[j + 1]; ++e) {
        const int32_t packed = a.child[e];
        const int64_t sp = packed >> SH;
        const int m = packed & (KP - 1);
        const double z = (double)a.xibar_in[a.n0 + sp] / (double)a.sigma[sp];
        acc = fma(-(double)a.b[((sp >> 6) * KP + m) * kTile + (sp & 63)], z, acc);
    }
    a.vbar_out[j] = (TS)acc;
}

// ---- dense block, inverse part: t0 = L0^-T xibar0, vbar_out[0:n0] += t0
template <typename TS>
__global__ __launch_bounds__(VECCHIA_N0MAX) void adj_dense_inverse_kernel(AdjArgs<TS> a) {
    __shared__ double t[VECCHIA_N0MAX];
    const int i = threadIdx.x;
    const int n0 = a.n0;
    double ri = i < n0 ? (double)a.xibar_in[i] : 0.0;
    for (int j = n0 - 1; j >= 0; --j) {
        if (i == j) t[j] = ri / a.l0[j * n0 + j];
        __syncthreads();
        if (i < j) ri = fma(-a.l0[j * n0 + i], t[j], ri);
    }
    if (i < n0) {
        a.t0[i] = t[i];
        a.vbar_out[i] = (TS)((double)a.vbar_out[i] + t[i]);
    }
}

// ---- per sparse point: theta contributions (double throughout)
template <typename TS, int K, int KIND>
__global__ __launch_bounds__(kBlock) void adj_theta_kernel(AdjArgs<TS> a) {
    constexpr int P = factor_lanes(VECCHIA_FP64, K);
    constexpr int R = K / P;
    constexpr int NA = P * R * (R + 1) / 2;
    constexpr int PTS = kBlock / P;
    const int tid = threadIdx.x;
    const int r = tid % P;
    const int64_t sp_raw = (int64_t)blockIdx.x * PTS + tid / P;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;
    const int64_t base = (sp >> 6) * (int64_t)K * kTile + (sp & 63);
    const int64_t s = a.n0 + sp;

    const double sig = (double)a.sigma[sp];
    double omega = a.vbar ? a.w[s] : 0.0;
    if (a.xibar_in) omega -= (double)a.xibar_in[s] / sig;
    const double sigma_bar = omega * (double)a.xi[s] + 2.0 * a.ldbar / sig;
    const double sbar = sigma_bar / (2.0 * sig);

    double c0[R], c1[R], c2[R];
    int ok[R];
    gather_rows<double, TS, K, P>(a.x, a.nbr, base, r, c0, c1, c2, ok);
    double bq[R], bbar[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        const int32_t j = a.nbr[base + (int64_t)(p * P + r) * kTile];
        bq[p] = (double)a.b[base + (int64_t)(p * P + r) * kTile];
        const double vj = (double)a.v[j >= 0 ? j : 0];   // unconditional load, selected below
        bbar[p] = j >= 0 ? omega * vj : 0.0;
    });

    double A[NA];
    assemble_kcc<double, K, P, KIND>(c0, c1, c2, ok, r, a.cov, A);
    double Dg[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        Dg[p] = ok[p] ? a.diag : 1.0;
    });
    double Inv[R];
    bool bad = false;
    double minpiv = 1.0;
    cholesky_kcc<double, K, P>(A, Dg, Inv, r, bad, minpiv);
    double u[R];
    static_for<0, R>([&](auto PI) { u[(int)PI] = bbar[(int)PI]; });
    lower_solve<double, K, P>(A, Inv, u, r);
    upper_solve<double, K, P>(A, Inv, u, r);

    const TS* xt = a.x + s * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];
    // Off the diagonals every covariance entry is kappa, whose sigma
    // derivative is 2 kappa / sigma: acc_k collects the kappa-weighted terms
    // and is scaled once at the end.
    double acc_k = 0.0, acc_l = 0.0;
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        double kap, dl;
        cov_and_dell<KIND>(sqdist3(c0[p], c1[p], c2[p], t0, t1, t2), a.cov, kap, dl);
        const double coef = ok[p] ? (u[p] - 2.0 * sbar * bq[p]) : 0.0;
        acc_k = fma(coef, kap, acc_k);
        acc_l = fma(coef, dl, acc_l);
    });
    // sum_{i,j} cw_i b_j dK_ij with cw_i = sbar b_i - u_i over the distinct
    // entries of the symmetric dK: the diagonal (dK_ii / dsigma = 2 sigma,
    // dK_ii / dell = 0) with weight cw_i b_i, each entry below it with
    // cw_i b_j + cw_j b_i.  For column q the lane takes its rows below q: its
    // row blocks after q's, and in q's block the lanes after q's.
    double cw[R];
    double acc_d = 0.0;
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        cw[p] = sbar * bq[p] - u[p];
        acc_d = fma(ok[p] ? cw[p] : 0.0, bq[p], acc_d);
    });
    static_for<0, K>([&](auto QI) {
        constexpr int q = QI, pq = q / P, rq = q % P;
        const double y0 = group_bcast<P, rq>(c0[pq]);
        const double y1 = group_bcast<P, rq>(c1[pq]);
        const double y2 = group_bcast<P, rq>(c2[pq]);
        const int okq = group_bcast<P, rq>(ok[pq]);
        const double bqq = group_bcast<P, rq>(bq[pq]);
        const double cwq = group_bcast<P, rq>(cw[pq]);
        static_for<pq, R>([&](auto PI) {
            constexpr int p = PI;
            double kap, dl;
            cov_and_dell<KIND>(sqdist3(c0[p], c1[p], c2[p], y0, y1, y2), a.cov, kap, dl);
            bool use = (ok[p] & okq) != 0;
            if constexpr (p == pq) use = use && r > rq;
            const double wgt = use ? fma(cw[p], bqq, cwq * bq[p]) : 0.0;
            acc_k = fma(wgt, kap, acc_k);
            acc_l = fma(wgt, dl, acc_l);
        });
    });
    double acc_s = fma(acc_k, 2.0 / a.sigma_amp, acc_d * (2.0 * a.sigma_amp));
    acc_s = group_sum<P>(acc_s);
    acc_l = group_sum<P>(acc_l);
    if (r == 0) acc_s = fma(sbar, 2.0 * a.sigma_amp, acc_s);   // dK_ii / dsigma
    if (!live || r != 0) acc_s = acc_l = 0.0;
    __shared__ double sh[2 * (kBlock / 64)];
    block_sum2(acc_s, acc_l, sh);
    if (tid == 0) {
        a.theta_part[2 * blockIdx.x] = acc_s;
        a.theta_part[2 * blockIdx.x + 1] = acc_l;
    }
}

// ---- dense block: xibar0 = L0^T w0 and the Cholesky adjoint contribution.
// kDenseLanes lanes serve each row (or column): lane u takes the entries
// l = u, u + 8, ... of every dot product and the group sums them in a fixed
// butterfly.  The two triangular solves walk L0 column by column from the
// last; column j is read from LDS while column j - 1 is being loaded.
constexpr int kDenseLanes = 8;
constexpr int kDenseThreads = VECCHIA_N0MAX * kDenseLanes;

template <typename TS, int KIND>
__global__ __launch_bounds__(kDenseThreads) void adj_dense_kernel(AdjArgs<TS> a) {
    constexpr int LD = VECCHIA_N0MAX + 1;
    constexpr int T = kDenseLanes;
    __shared__ double X[VECCHIA_N0MAX * LD];
    __shared__ double G[VECCHIA_N0MAX], Z[VECCHIA_N0MAX], H[VECCHIA_N0MAX];
    __shared__ double Lc[2][VECCHIA_N0MAX];     // one column of L0, double-buffered
    __shared__ double Pt[VECCHIA_N0MAX][3];     // coordinates of the dense block
    __shared__ double sh[2 * (kDenseThreads / 64)];
    const int tid = threadIdx.x;
    const int i = tid / T, u = tid % T;          // row (or column) i, lane u of its group
    const int n0 = a.n0;
    const bool row = i < n0;                     // the same for the whole group
    const double* L = a.l0;
    if (tid < n0) {
        double g = a.vbar ? a.w[tid] : 0.0;
        if (a.xibar_in) g -= a.t0[tid];
        G[tid] = g;
        Z[tid] = (double)a.xi[tid];
        Pt[tid][0] = (double)a.x[tid * 3];
        Pt[tid][1] = (double)a.x[tid * 3 + 1];
        Pt[tid][2] = (double)a.x[tid * 3 + 2];
        Lc[(n0 - 1) & 1][tid] = L[tid * n0 + n0 - 1];
    }
    __syncthreads();
    // h = L0^T g and xibar0 = L0^T w0 (column i of L0)
    {
        double h = 0.0, xb = 0.0;
        if (row) {
            for (int m = i + u; m < n0; m += T) {
                const double l = L[m * n0 + i];
                h = fma(l, G[m], h);
                if (a.vbar) xb = fma(l, a.w[m], xb);
            }
        }
        h = group_sum<T>(h);
        xb = group_sum<T>(xb);
        if (row && u == 0) {
            H[i] = h;
            if (a.vbar) a.xibar[i] = (TS)xb;
        }
    }
    __syncthreads();
    // X = M L0^-1, row i: x L0 = m  (backward over columns)
    for (int j = n0 - 1; j >= 0; --j) {
        const double nxt = (j > 0 && tid < n0) ? L[tid * n0 + j - 1] : 0.0;
        const double* lc = Lc[j & 1];
        double part = 0.0;
        if (row)
            for (int l = j + 1 + u; l < n0; l += T) part = fma(X[i * LD + l], lc[l], part);
        part = group_sum<T>(part);
        if (row && u == 0) {
            const double m = j < i ? H[i] * Z[j] : (j == i ? 0.5 * H[i] * Z[i] + a.ldbar : 0.0);
            X[i * LD + j] = (m - part) / lc[j];
        }
        if (j > 0 && tid < n0) Lc[(j - 1) & 1][tid] = nxt;
        __syncthreads();
    }
    // Y = L0^-T X, column i: L0^T y = x  (backward over rows), in place
    if (tid < n0) Lc[(n0 - 1) & 1][tid] = L[tid * n0 + n0 - 1];
    __syncthreads();
    for (int rr = n0 - 1; rr >= 0; --rr) {
        const double nxt = (rr > 0 && tid < n0) ? L[tid * n0 + rr - 1] : 0.0;
        const double* lc = Lc[rr & 1];
        double part = 0.0;
        if (row)
            for (int l = rr + 1 + u; l < n0; l += T) part = fma(lc[l], X[l * LD + i], part);
        part = group_sum<T>(part);
        if (row && u == 0) X[rr * LD + i] = (X[rr * LD + i] - part) / lc[rr];
        if (rr > 0 && tid < n0) Lc[(rr - 1) & 1][tid] = nxt;
        __syncthreads();
    }
    double acc_s = 0.0, acc_l = 0.0;
    if (row) {
        const double p0 = Pt[i][0], p1 = Pt[i][1], p2 = Pt[i][2];
        for (int j = u; j < n0; j += T) {
            double kap, dl;
            cov_and_dell<KIND>(sqdist3(p0, p1, p2, Pt[j][0], Pt[j][1], Pt[j][2]), a.cov, kap, dl);
            const double y = X[i * LD + j];
            acc_s = fma(y, i == j ? 2.0 * a.sigma_amp : 2.0 * kap / a.sigma_amp, acc_s);
            acc_l = fma(y, i == j ? 0.0 : dl, acc_l);
        }
    }
    block_sum2(acc_s, acc_l, sh);
    if (tid == 0) {
        a.theta_dense[0] = acc_s;
        a.theta_dense[1] = acc_l;
    }
    // coordinates: K0_bar = sym(Y) acts on both points of every entry, so
    // point i receives sum_j (Y_ij + Y_ji) kappa'(r)/r (x_i - x_j)
    if (a.xgrad) {
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
        if (row) {
            const double p0 = Pt[i][0], p1 = Pt[i][1], p2 = Pt[i][2];
            for (int j = u; j < n0; j += T) {
                const double q0 = Pt[j][0], q1 = Pt[j][1], q2 = Pt[j][2];
                double kap, ds;
                cov_and_dr<KIND>(sqdist3(p0, p1, p2, q0, q1, q2), a.cov, kap, ds);
                const double wgt = j == i ? 0.0 : (X[i * LD + j] + X[j * LD + i]) * ds;
                g0 = fma(wgt, p0 - q0, g0);
                g1 = fma(wgt, p1 - q1, g1);
                g2 = fma(wgt, p2 - q2, g2);
            }
        }
        g0 = group_sum<T>(g0);
        g1 = group_sum<T>(g1);
        g2 = group_sum<T>(g2);
        if (row && u == 0) {
            a.xgrad[i * 3] = g0;
            a.xgrad[i * 3 + 1] = g1;
            a.xgrad[i * 3 + 2] = g2;
        }
    }
}

// ---- theta = sum of the per-block partials (compensated, fixed order) + dense
__global__ __launch_bounds__(1024) void adj_theta_reduce_kernel(const double* __restrict__ part, int64_t nblocks,
                                                                const double* __restrict__ dense,
                                                                double* __restrict__ out) {
    __shared__ double S[2][1024], C[2][1024];
    double s[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
    for (int64_t b = threadIdx.x; b < nblocks; b += 1024)
        for (int t = 0; t < 2; ++t) {
            const double x = part[2 * b + t];
            const double y = s[t] + x;
            c[t] += fabs(s[t]) >= fabs(x) ? (s[t] - y) + x : (x - y) + s[t];
            s[t] = y;
        }
    for (int t = 0; t < 2; ++t) {
        S[t][threadIdx.x] = s[t];
        C[t][threadIdx.x] = c[t];
    }
    __syncthreads();
    for (int stride = 512; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
            for (int t = 0; t < 2; ++t) {
                const double x = S[t][threadIdx.x + stride];
                const double y = S[t][threadIdx.x] + x;
                const double e = fabs(S[t][threadIdx.x]) >= fabs(x) ? (S[t][threadIdx.x] - y) + x
                                                                    : (x - y) + S[t][threadIdx.x];
                S[t][threadIdx.x] = y;
                C[t][threadIdx.x] += C[t][threadIdx.x + stride] + e;
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int t = 0; t < 2; ++t) out[t] = (S[t][0] + C[t][0]) + dense[t];
}

template <typename TS, int KP, int KIND>
static hipError_t backward_t(const BackwardLaunch& p, hipStream_t s) {
    AdjArgs<TS> a;
    a.x = static_cast<const TS*>(p.x);
    a.nbr = p.nbr;
    a.child_ptr = p.child_ptr;
    a.child = p.child;
    a.b = static_cast<const TS*>(p.b);
    a.sigma = static_cast<const TS*>(p.sigma);
    a.l0 = p.l0;
    a.xi = static_cast<const TS*>(p.xi);
    a.v = static_cast<const TS*>(p.v);
    a.vbar = static_cast<const TS*>(p.vbar);
    a.xibar_in = static_cast<const TS*>(p.xibar_in);
    a.w = static_cast<double*>(p.w);
    a.xibar = static_cast<TS*>(p.xibar);
    a.vbar_out = static_cast<TS*>(p.vbar_out);
    a.t0 = p.t0;
    a.theta_part = p.theta_part;
    a.theta_dense = p.theta_dense;
    a.theta_out = p.theta_out;
    a.n = p.n;
    a.ns = p.ns;
    a.n0 = p.n0;
    a.kp = KP;
    a.ldbar = p.ldbar;
    a.sigma_amp = p.kern.sigma;
    a.diag = p.kern.sigma * p.kern.sigma + p.kern.nugget;
    a.cov = make_cov<double>(p.kern);
    constexpr int P = factor_lanes(VECCHIA_FP64, KP);
    a.nblocks = (p.ns + kBlock / P - 1) / (kBlock / P);
    hipError_t e = hipSuccess;
    if (p.vbar) {
        for (int l = p.n_levels; l >= 0; --l) {
            const int64_t j0 = l == 0 ? 0 : p.level_ptr[l], j1 = l == 0 ? p.n0 : p.level_ptr[l + 1];
            if (j1 <= j0) continue;
            if ((e = launch_adj_sweep<TS, KP>(a, j0, j1, s)) != hipSuccess) return e;
        }
    }
    if (p.xibar_in) {
        hipLaunchKernelGGL((adj_inverse_kernel<TS, KP>), dim3((unsigned)((p.n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((adj_dense_inverse_kernel<TS>), dim3(1), dim3(VECCHIA_N0MAX), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.nblocks > 0) {
        if constexpr (KP == 64) {
            if ((e = launch_adj_theta_wide<TS>(a, KIND, s)) != hipSuccess) return e;
        } else {
            hipLaunchKernelGGL((adj_theta_kernel<TS, KP, KIND>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL((adj_dense_kernel<TS, KIND>), dim3(1), dim3(kDenseThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(adj_theta_reduce_kernel, dim3(1), dim3(1024), 0, s, a.theta_part, a.nblocks, a.theta_dense,
                       a.theta_out);
    return hipGetLastError();
}

// ---- coordinates (at a fixed graph), per sparse point i: with u, sbar and
// b as in adj_theta_kernel, the cotangents k_bar_p = u_p - 2 sbar b_p of
// k_ci and K_bar_pq = sbar b_p b_q - u_p b_q of K_cc act through
// g(x_p, x_q) = kappa'(r)/r (x_p - x_q) = d kappa(|x_p - x_q|) / d x_p:
//   x_bar_i      -= sum_p k_bar_p g(x_p, x_i)       (written here)
//   x_bar_{c(p)} += k_bar_p g(x_p, x_i) + sum_q (K_bar_pq + K_bar_qp) g(x_p, x_q)
// the latter stored per row entry (tiled like b, a record of 3 doubles each)
// and summed into each neighbour by adj_x_gather_kernel over the children
// lists, in a fixed order.
template <typename TS, int K, int KIND>
__global__ __launch_bounds__(kBlock) void adj_x_kernel(AdjArgs<TS> a, double* __restrict__ contrib) {
    constexpr int P = factor_lanes(VECCHIA_FP64, K);
    constexpr int R = K / P;
    constexpr int NA = P * R * (R + 1) / 2;
    constexpr int PTS = kBlock / P;
    const int tid = threadIdx.x;
    const int r = tid % P;
    const int64_t sp_raw = (int64_t)blockIdx.x * PTS + tid / P;
    const bool live = sp_raw < a.ns;
    const int64_t sp = live ? sp_raw : a.ns - 1;
    const int64_t base = (sp >> 6) * (int64_t)K * kTile + (sp & 63);
    const int64_t s = a.n0 + sp;

    const double sig = (double)a.sigma[sp];
    double omega = a.vbar ? a.w[s] : 0.0;
    if (a.xibar_in) omega -= (double)a.xibar_in[s] / sig;
    const double sigma_bar = omega * (double)a.xi[s] + 2.0 * a.ldbar / sig;
    const double sbar = sigma_bar / (2.0 * sig);

    double c0[R], c1[R], c2[R];
    int ok[R];
    gather_rows<double, TS, K, P>(a.x, a.nbr, base, r, c0, c1, c2, ok);
    double bq[R], bbar[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        const int32_t j = a.nbr[base + (int64_t)(p * P + r) * kTile];
        bq[p] = (double)a.b[base + (int64_t)(p * P + r) * kTile];
        const double vj = (double)a.v[j >= 0 ? j : 0];   // unconditional load, selected below
        bbar[p] = j >= 0 ? omega * vj : 0.0;
    });

    double A[NA];
    assemble_kcc<double, K, P, KIND>(c0, c1, c2, ok, r, a.cov, A);
    double Dg[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        Dg[p] = ok[p] ? a.diag : 1.0;
    });
    double Inv[R];
    bool bad = false;
    double minpiv = 1.0;
    cholesky_kcc<double, K, P>(A, Dg, Inv, r, bad, minpiv);
    double u[R];
    static_for<0, R>([&](auto PI) { u[(int)PI] = bbar[(int)PI]; });
    lower_solve<double, K, P>(A, Inv, u, r);
    upper_solve<double, K, P>(A, Inv, u, r);

    const TS* xt = a.x + s * 3;
    const double t0 = (double)xt[0], t1 = (double)xt[1], t2 = (double)xt[2];
    double own0 = 0.0, own1 = 0.0, own2 = 0.0;
    double g0[R], g1[R], g2[R];
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        double kap, ds;
        cov_and_dr<KIND>(sqdist3(c0[p], c1[p], c2[p], t0, t1, t2), a.cov, kap, ds);
        const double w = ok[p] ? (u[p] - 2.0 * sbar * bq[p]) * ds : 0.0;
        g0[p] = w * (c0[p] - t0);
        g1[p] = w * (c1[p] - t1);
        g2[p] = w * (c2[p] - t2);
        own0 -= g0[p];
        own1 -= g1[p];
        own2 -= g2[p];
    });
    // Each unordered pair once: for column q the lane takes its rows below q
    // (its row blocks from q's block down, in q's own block the lanes after
    // q's); the pair's term goes to the row with + and to row q with -, the
    // latter summed over the group and added by q's lane.
    static_for<0, K>([&](auto QI) {
        constexpr int q = QI, pq = q / P, rq = q % P;
        const double y0 = group_bcast<P, rq>(c0[pq]);
        const double y1 = group_bcast<P, rq>(c1[pq]);
        const double y2 = group_bcast<P, rq>(c2[pq]);
        const int okq = group_bcast<P, rq>(ok[pq]);
        const double bqq = group_bcast<P, rq>(bq[pq]);
        const double uq = group_bcast<P, rq>(u[pq]);
        double h0 = 0.0, h1 = 0.0, h2 = 0.0;
        static_for<pq, R>([&](auto PI) {
            constexpr int p = PI;
            double kap, ds;
            cov_and_dr<KIND>(sqdist3(c0[p], c1[p], c2[p], y0, y1, y2), a.cov, kap, ds);
            bool use = (ok[p] & okq) != 0;
            if constexpr (p == pq) use = use && r > rq;
            const double w = use ? (2.0 * sbar * bq[p] * bqq - u[p] * bqq - uq * bq[p]) * ds : 0.0;
            const double d0 = w * (c0[p] - y0), d1 = w * (c1[p] - y1), d2 = w * (c2[p] - y2);
            g0[p] += d0;
            g1[p] += d1;
            g2[p] += d2;
            h0 -= d0;
            h1 -= d1;
            h2 -= d2;
        });
        h0 = group_sum<P>(h0);
        h1 = group_sum<P>(h1);
        h2 = group_sum<P>(h2);
        if (r == rq) {
            g0[pq] += h0;
            g1[pq] += h1;
            g2[pq] += h2;
        }
    });
    own0 = group_sum<P>(own0);
    own1 = group_sum<P>(own1);
    own2 = group_sum<P>(own2);
    if (!live) return;
    static_for<0, R>([&](auto PI) {
        constexpr int p = PI;
        double* rec = contrib + 3 * (base + (int64_t)(p * P + r) * kTile);
        rec[0] = g0[p];
        rec[1] = g1[p];
        rec[2] = g2[p];
    });
    if (r == 0) {
        a.xgrad[s * 3] = own0;
        a.xgrad[s * 3 + 1] = own1;
        a.xgrad[s * 3 + 2] = own2;
    }
}

// x_bar_j += the stored row contributions of every child entry of j, in the
// children lists' (ascending) order.
template <int KP>
__global__ __launch_bounds__(kBlock) void adj_x_gather_kernel(const int64_t* __restrict__ child_ptr,
                                                              const int32_t* __restrict__ child,
                                                              const double* __restrict__ contrib,
                                                              double* __restrict__ xgrad, int64_t n) {
    constexpr int SH = KP == 8 ? 3 : (KP == 16 ? 4 : (KP == 32 ? 5 : 6));
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    double g0 = xgrad[j * 3], g1 = xgrad[j * 3 + 1], g2 = xgrad[j * 3 + 2];
#pragma unroll 4
    for (int64_t e = child_ptr[j]; e < child_ptr[j + 1]; ++e) {
        const int32_t packed = child[e];
        const int64_t sp = packed >> SH;
        const int m = packed & (KP - 1);
        const double* rec = contrib + 3 * (((sp >> 6) * KP + m) * kTile + (sp & 63));
        g0 += rec[0];
        g1 += rec[1];
        g2 += rec[2];
    }
    xgrad[j * 3] = g0;
    xgrad[j * 3 + 1] = g1;
    xgrad[j * 3 + 2] = g2;
}

template <typename TS, int KP, int KIND>
static hipError_t backward_x_t(const BackwardLaunch& p, double* xgrad, double* contrib, hipStream_t s) {
    AdjArgs<TS> a;
    a.x = static_cast<const TS*>(p.x);
    a.nbr = p.nbr;
    a.child_ptr = p.child_ptr;
    a.child = p.child;
    a.b = static_cast<const TS*>(p.b);
    a.sigma = static_cast<const TS*>(p.sigma);
    a.l0 = p.l0;
    a.xi = static_cast<const TS*>(p.xi);
    a.v = static_cast<const TS*>(p.v);
    a.vbar = static_cast<const TS*>(p.vbar);
    a.xibar_in = static_cast<const TS*>(p.xibar_in);
    a.w = static_cast<double*>(p.w);
    a.xibar = static_cast<TS*>(p.xibar);
    a.vbar_out = static_cast<TS*>(p.vbar_out);
    a.t0 = p.t0;
    a.theta_part = p.theta_part;
    a.theta_dense = p.theta_dense;
    a.theta_out = p.theta_out;
    a.n = p.n;
    a.ns = p.ns;
    a.n0 = p.n0;
    a.kp = KP;
    a.ldbar = p.ldbar;
    a.sigma_amp = p.kern.sigma;
    a.diag = p.kern.sigma * p.kern.sigma + p.kern.nugget;
    a.cov = make_cov<double>(p.kern);
    a.xgrad = xgrad;
    constexpr int P = factor_lanes(VECCHIA_FP64, KP);
    a.nblocks = (p.ns + kBlock / P - 1) / (kBlock / P);
    hipError_t e = hipSuccess;
    if (p.vbar) {
        for (int l = p.n_levels; l >= 0; --l) {
            const int64_t j0 = l == 0 ? 0 : p.level_ptr[l], j1 = l == 0 ? p.n0 : p.level_ptr[l + 1];
            if (j1 <= j0) continue;
            if ((e = launch_adj_sweep<TS, KP>(a, j0, j1, s)) != hipSuccess) return e;
        }
    }
    if (p.xibar_in) {
        hipLaunchKernelGGL((adj_inverse_kernel<TS, KP>), dim3((unsigned)((p.n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((adj_dense_inverse_kernel<TS>), dim3(1), dim3(VECCHIA_N0MAX), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.nblocks > 0) {
        if constexpr (KP == 64) {
            if ((e = launch_adj_x_wide<TS>(a, KIND, contrib, s)) != hipSuccess) return e;
        } else {
            hipLaunchKernelGGL((adj_x_kernel<TS, KP, KIND>), dim3((unsigned)a.nblocks), dim3(kBlock), 0, s, a,
                               contrib);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL((adj_dense_kernel<TS, KIND>), dim3(1), dim3(kDenseThreads), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((adj_x_gather_kernel<KP>), dim3((unsigned)((p.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       p.child_ptr, p.child, contrib, xgrad, p.n);
    return hipGetLastError();
}

template <typename TS, int KP>
static hipError_t backward_x_kind(const BackwardLaunch& p, double* xgrad, double* contrib, hipStream_t s) {
    switch (p.kern.kind) {
        case 0: return backward_x_t<TS, KP, 0>(p, xgrad, contrib, s);
        case 1: return backward_x_t<TS, KP, 1>(p, xgrad, contrib, s);
        case 2: return backward_x_t<TS, KP, 2>(p, xgrad, contrib, s);
        case 3: return backward_x_t<TS, KP, 3>(p, xgrad, contrib, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename TS>
static hipError_t backward_x_width(const BackwardLaunch& p, double* xgrad, double* contrib, hipStream_t s) {
    switch (p.kp) {
        case 8: return backward_x_kind<TS, 8>(p, xgrad, contrib, s);
        case 16: return backward_x_kind<TS, 16>(p, xgrad, contrib, s);
        case 32: return backward_x_kind<TS, 32>(p, xgrad, contrib, s);
        case 64: return backward_x_kind<TS, 64>(p, xgrad, contrib, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward_x(const BackwardLaunch& p, double* xgrad, double* contrib, hipStream_t s) {
    return p.precision == VECCHIA_FP32 ? backward_x_width<float>(p, xgrad, contrib, s)
                                       : backward_x_width<double>(p, xgrad, contrib, s);
}

template <typename TS, int KP>
static hipError_t backward_kind(const BackwardLaunch& p, hipStream_t s) {
    switch (p.kern.kind) {
        case 0: return backward_t<TS, KP, 0>(p, s);
        case 1: return backward_t<TS, KP, 1>(p, s);
        case 2: return backward_t<TS, KP, 2>(p, s);
        case 3: return backward_t<TS, KP, 3>(p, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename TS>
static hipError_t backward_width(const BackwardLaunch& p, hipStream_t s) {
    switch (p.kp) {
        case 8: return backward_kind<TS, 8>(p, s);
        case 16: return backward_kind<TS, 16>(p, s);
        case 32: return backward_kind<TS, 32>(p, s);
        case 64: return backward_kind<TS, 64>(p, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward(const BackwardLaunch& p, hipStream_t s) {
    return p.precision == VECCHIA_FP32 ? backward_width<float>(p, s) : backward_width<double>(p, s);
}

}  // namespace vk
