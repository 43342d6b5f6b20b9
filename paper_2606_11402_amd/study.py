"""Order and accuracy study of the method (Fig. 1, centre and right).

* Batch sizes: the parallel batches (depth levels, Sec. 2.2 "Batch
  construction") of the bit-reversed tree order for a point cloud, from the
  host graph build.
* Accuracy: the Kullback-Leibler divergence of the Vecchia approximation
  N(0, K~) from the exact Gaussian process N(0, K),
      KL = 1/2 [ tr(K~^-1 K) - N + log det K~ - log det K ],
  with K~ = F F^T and F = (I - B)^-1 D (Sec. 2.1: the approximation's
  precision is sparse).  K~^-1 = (I - B)^T D^-2 (I - B), so
      tr(K~^-1 K) = || D^-1 (I - B) L_K ||_F^2,   K = L_K L_K^T,
  where the rows of D^-1 (I - B) are (e_i - b_i . e_c(i)) / sigma_i for the
  sparse points and L0^-1 for the dense block.  b, sigma, L0 and log det K~
  come from the GPU factor (vecchia_factor, vecchia_logdet, FP64); K and its
  Cholesky factor are formed densely in FP64 on the host, which limits the
  study to N of order 10^4 (the paper's setting).

The paper's figure data are absent, so these values are not compared with
printed numbers.  Usage:

    python -m paper_2606_11402_amd.study            # N = 10^4 unit Gaussian, n0 = 50

prints one JSON line.
"""
import argparse
import json
import time

import numpy as np
import scipy.sparse
import torch

from .vecchia import EXP, FP64, M32, M52, SE, Factor, Graph, KernelParams

KIND_NAMES = {EXP: "matern-1/2", M32: "matern-3/2", M52: "matern-5/2", SE: "matern-inf (squared exponential)"}


def batch_sizes(graph):
    """Sizes of the parallel batches 1..L (the dense block excluded)."""
    lp = np.asarray(graph.level_ptr, dtype=np.int64)
    return np.diff(lp[1:])


def kernel_matrix(xs, kern):
    """Dense K(xs, xs) with the nugget on the diagonal (host, FP64)."""
    d = xs[:, None, :] - xs[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    s2 = kern.sigma * kern.sigma
    if kern.kind == EXP:
        k = s2 * np.exp(-r / kern.ell)
    elif kern.kind == M32:
        a = np.sqrt(3.0) * r / kern.ell
        k = s2 * (1.0 + a) * np.exp(-a)
    elif kern.kind == M52:
        a = np.sqrt(5.0) * r / kern.ell
        k = s2 * (1.0 + a + a * a / 3.0) * np.exp(-a)
    elif kern.kind == SE:
        k = s2 * np.exp(-(r * r) / (2.0 * kern.ell * kern.ell))
    else:
        raise ValueError(kern.kind)
    k[np.diag_indices_from(k)] += kern.nugget
    return k


def precision_factor(graph, b_dev, sigma, l0):
    """D^-1 (I - B) in storage order as a CSR matrix, from the device rows
    (tiled neighbour indices and coefficients, same order) and L0."""
    n, n0, kp = graph.n, graph.n0, graph.kp
    ns = n - n0
    nbr = graph.nbr(1).reshape(graph.ntiles, kp, 64).transpose(0, 2, 1).reshape(-1, kp)[:ns]
    b = np.asarray(b_dev, dtype=np.float64)[:ns]
    inv_l0 = np.linalg.inv(np.tril(l0))                          # dense block rows: L0^-1
    r0, c0 = np.nonzero(np.tril(np.ones((n0, n0))))
    rows = [r0, np.arange(n0, n)]
    cols = [c0, np.arange(n0, n)]
    vals = [inv_l0[r0, c0], 1.0 / sigma]
    ok = nbr >= 0
    rr = np.repeat(np.arange(n0, n), kp).reshape(ns, kp)
    rows.append(rr[ok])
    cols.append(nbr[ok].astype(np.int64))
    vals.append((-b / sigma[:, None])[ok])
    return scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def exact_cholesky(x, kern):
    """Cholesky factor of the exact K for the points in input order, and
    log det K (host, FP64)."""
    lk = np.linalg.cholesky(kernel_matrix(np.asarray(x, dtype=np.float64), kern))
    return lk, 2.0 * float(np.sum(np.log(np.diag(lk))))


def kl_divergence(x, k, n0, kern, device="cuda:0", exact=None):
    """KL(N(0, K) || N(0, K~)) for the points x (input order) with k
    neighbours and a dense block of n0.  exact = exact_cholesky(x, kern)
    may be passed to reuse it across k.  tr(M K M^T) with M = D^-1 (I - B)
    in storage order equals || M[:, pos] L ||_F^2 with L the Cholesky factor
    of K in input order and pos[q] the storage position of input point q.
    Returns (kl, graph, details)."""
    g = Graph(x, k, n0)
    dg = g.to_device(FP64, device)
    fac = Factor(dg, KernelParams(kern.kind, kern.sigma, kern.ell, kern.nugget))
    fac.status()
    ld_tilde = fac.logdet().item()
    b_dev, sigma = fac.coefficients()
    l0 = fac._ws_slice("L0").cpu().numpy().copy()
    lk, ld_k = exact if exact is not None else exact_cholesky(x, kern)
    pos = np.empty(g.n, dtype=np.int64)
    pos[g.order] = np.arange(g.n)
    m = precision_factor(g, b_dev, sigma.astype(np.float64), l0)[:, pos]
    y = m @ lk
    tr = float(np.sum(y * y))
    kl = 0.5 * (tr - g.n + ld_tilde - ld_k)
    return kl, g, {"trace": tr, "logdet_vecchia": ld_tilde, "logdet_exact": ld_k}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--n0", type=int, default=50)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--ell", type=float, default=1.0)
    ap.add_argument("--nugget", type=float, default=1e-8)
    ap.add_argument("--ks", default="1,2,4,8,16,32,64")
    ap.add_argument("--level-ns", default="10000,100000,1000000,10000000")
    args = ap.parse_args()
    rng = np.random.default_rng(args.seed)
    x = rng.standard_normal((args.n, 3))                          # unit Gaussian in 3-D
    out = {"n": args.n, "n0": args.n0, "points": "unit Gaussian in 3-D", "seed": args.seed, "ell": args.ell,
           "sigma": 1.0, "nugget": args.nugget}
    g = Graph(x, 16, args.n0)
    bs = batch_sizes(g)
    out["batches_k16"] = {"levels": int(g.n_levels), "largest": int(bs.max()), "median": float(np.median(bs)),
                          "sizes": bs.tolist()}
    levels = {}
    for nn in [int(s) for s in args.level_ns.split(",") if s]:
        xx = np.random.default_rng(args.seed + 1).standard_normal((nn, 3))
        for kk in (8, 16, 32):
            gg = Graph(xx, kk, args.n0)
            levels["n=%d,k=%d" % (nn, kk)] = int(gg.n_levels)
    out["levels_vs_n"] = levels
    kl = {}
    for kind in (EXP, M32, M52, SE):
        kern = KernelParams(kind, 1.0, args.ell, args.nugget)
        exact = exact_cholesky(x, kern)
        row = {}
        for kk in [int(s) for s in args.ks.split(",") if s]:
            t = time.time()
            val, _, det = kl_divergence(x, kk, args.n0, kern, exact=exact)
            row[kk] = val
            print("[study] %s k=%d KL=%.4e (%.1fs)" % (KIND_NAMES[kind], kk, val, time.time() - t), flush=True)
        kl[KIND_NAMES[kind]] = row
    out["kl_vs_k"] = kl
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
